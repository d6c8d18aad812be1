// Row-update kernels shared by the compressed multiplicative updates
// (Alg. 2 with the semi-NMF rule of Ding et al. 2010, Eq. 8) and by the
// uncompressed comparators (Alg. 3 and Alg. 2 with L = I, R = I).
//
// One launch updates the rows of one factor (X, or Y^T) and accumulates the
// block's partial sum for the next half-step:
//   z      = B1[i] C                (compressed: N = Ac Yc^T or N2 = B^T Xh)
//          = P[i]                   (uncompressed: a row of A Y^T / A^T X)
//   MU:    F[i] <- F[i] o sqrt((z+ + F[i] G-) / (z- + F[i] G+ + eps))
//   ADMM:  xt = (z + pen F[i] - Mu[i]) Minv;  F[i] = max(xt + Mu[i]/pen, 0);
//          Mu[i] += xi pen (xt - F[i])
//   partial: B2[i]^T F_new[i]  (k2 x r)   or the Gram out[i]^T out[i] (r x r)
//   optional: out[i] (F_new for MU, xt for ADMM) written to an operand
//   buffer for the next streaming pass.
#include "cnmf_internal.hpp"
#include "small_dense.hpp"

namespace cnmf {

constexpr int kRowCh = 16;   // rows per sweep: nr * ceil(r / 4) <= 256 work items

template <typename T>
__global__ __launch_bounds__(256) void nmf_row_kernel(RowArgs a) {
  const int tid = threadIdx.x;
  const int r = a.r, k1 = a.k1;
  const int k2 = a.B2 ? a.k2 : r;
  const int ldr = r + 1;
  const T* __restrict__ B1 = (const T*)a.B1;
  const T* __restrict__ B2 = (const T*)a.B2;
  T* __restrict__ F = (T*)a.F;
  T* __restrict__ Mu = (T*)a.Mu;
  T* __restrict__ Op = (T*)a.Op;
  extern __shared__ double sm[];
  double* cs = sm;                       // k1 x r (C) when compressed
  double* gp = cs + (a.C ? k1 * r : 0);  // r x r (G+ or Minv)
  double* gm = gp + r * r;               // r x r (G-)
  double* zs = gm + r * r;               // kRowCh x ldr: z, then the row outputs
  double* fs = zs + kRowCh * ldr;        // kRowCh x ldr: F rows, then F_new
  double* ms = fs + kRowCh * ldr;        // kRowCh x ldr: Mu rows
  double* b2s = ms + kRowCh * ldr;       // kRowCh x (k2 + 1)
  if (a.C)
    staged_copy<8>(k1 * r, tid, 256, [&](int e) { return a.C[e]; }, [&](int e, double v) { cs[e] = v; });
  if (a.method == 0) {
    staged_copy<8>(r * r, tid, 256, [&](int e) { return a.Gp[e]; }, [&](int e, double v) { gp[e] = v; });
    staged_copy<8>(r * r, tid, 256, [&](int e) { return a.Gm[e]; }, [&](int e, double v) { gm[e] = v; });
  } else if (a.method == 1) {
    staged_copy<8>(r * r, tid, 256, [&](int e) { return a.Minv[e]; }, [&](int e, double v) { gp[e] = v; });
  }
  const int ta = tid >> 4, tb = tid & 15;
  double acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const int i0 = blockIdx.x * a.rows_per_block;
  const int i1 = min(a.rows, i0 + a.rows_per_block);
  const int rq = (r + 3) / 4;
  // work item of this thread within a sweep: (row rr, columns c0..c0+3)
  const int my_rr = tid / rq, my_c0 = 4 * (tid - (tid / rq) * rq);
  for (int base = i0; base < i1; base += kRowCh) {
    const int nr = min(kRowCh, i1 - base);
    const bool have = my_rr < nr;
    __syncthreads();
    {
      const bool zb = !a.C && a.method != 2;
      struct V3 {
        double f, m, z;
      };
      staged_copy<4>(
          nr * r, tid, 256,
          [&](int e) {
            const int rr = e / r, c = e - rr * r;
            const int64_t off = (int64_t)(base + rr) * a.ldf + c;
            return V3{(double)F[off], Mu ? (double)Mu[off] : 0.0,
                      zb ? (double)B1[(int64_t)(base + rr) * a.ldb1 + c] : 0.0};
          },
          [&](int e, V3 v) {
            const int rr = e / r, c = e - rr * r;
            fs[rr * ldr + c] = v.f;
            ms[rr * ldr + c] = v.m;
            if (zb) zs[rr * ldr + c] = v.z;
          });
    }
    if (B2)
      staged_copy<8>(
          nr * k2, tid, 256, [&](int e) { const int rr = e / k2, c = e - rr * k2;
            return (double)B2[(int64_t)(base + rr) * a.ldb2 + c]; },
          [&](int e, double v) { const int rr = e / k2, c = e - rr * k2; b2s[rr * (k2 + 1) + c] = v; });
    __syncthreads();
    if (a.C && a.method != 2) {
      // z = B1[i] C
      if (have) {
        const T* brow = B1 + (int64_t)(base + my_rr) * a.ldb1;
        double s[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int l = 0; l < k1; ++l) {
          const double b = (double)brow[l];
#pragma unroll
          for (int u = 0; u < 4; ++u) s[u] = fma(b, cs[l * r + min(my_c0 + u, r - 1)], s[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (my_c0 + u < r) zs[my_rr * ldr + my_c0 + u] = s[u];
      }
      __syncthreads();
    }
    double fn[4] = {0, 0, 0, 0}, mn[4] = {0, 0, 0, 0}, out[4] = {0, 0, 0, 0};
    if (a.method != 2 && have) {
      const double* f = fs + my_rr * ldr;
      const double* z = zs + my_rr * ldr;
      const double* mu = ms + my_rr * ldr;
      if (a.method == 0) {
        double sp[4] = {0, 0, 0, 0}, sq[4] = {0, 0, 0, 0};
#pragma unroll 2
        for (int l = 0; l < r; ++l) {
          const double fl = f[l];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int c = min(my_c0 + u, r - 1);
            sp[u] = fma(fl, gp[l * r + c], sp[u]);
            sq[u] = fma(fl, gm[l * r + c], sq[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = my_c0 + u;
          if (c < r) {
            const double zc = z[c];
            const double zp = 0.5 * (fabs(zc) + zc), zm = 0.5 * (fabs(zc) - zc);
            fn[u] = f[c] * sqrt((zp + sq[u]) / (zm + sp[u] + a.eps));
            out[u] = fn[u];
          }
        }
      } else {
        double xt[4] = {0, 0, 0, 0};
#pragma unroll 2
        for (int l = 0; l < r; ++l) {
          const double rhs = z[l] + a.pen * f[l] - mu[l];
#pragma unroll
          for (int u = 0; u < 4; ++u) xt[u] = fma(rhs, gp[l * r + min(my_c0 + u, r - 1)], xt[u]);
        }
        const double ipen = 1.0 / a.pen, xpen = a.xi * a.pen;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = my_c0 + u;
          if (c < r) {
            const double t = xt[u] + mu[c] * ipen;
            fn[u] = t > 0.0 ? t : 0.0;
            mn[u] = mu[c] + xpen * (xt[u] - fn[u]);
            out[u] = xt[u];
          }
        }
      }
    }
    __syncthreads();
    if (a.method != 2 && have) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = my_c0 + u;
        if (c < r) {
          fs[my_rr * ldr + c] = fn[u];
          zs[my_rr * ldr + c] = out[u];
          const int64_t off = (int64_t)(base + my_rr) * a.ldf + c;
          F[off] = (T)fn[u];
          if (Mu) Mu[off] = (T)mn[u];
          if (Op) Op[(int64_t)(base + my_rr) * a.ldop + c] = (T)out[u];
        }
      }
    }
    __syncthreads();
    // partial sums over the staged rows: B2^T (new F), or the Gram of the
    // row outputs (the operand rows: new F for MU, xt for ADMM; for the
    // initial partial (method 2) the rows of F themselves)
    const double* wsrc = (B2 || a.method == 2) ? fs : zs;
    for (int rr = 0; rr < nr; ++rr) {
      double w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = tb + 16 * j;
        w[j] = c < r ? wsrc[rr * ldr + c] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int ai = ta + 16 * i;
        if (ai < k2) {
          const double b = B2 ? b2s[rr * (k2 + 1) + ai] : wsrc[rr * ldr + ai];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(b, w[j], acc[i][j]);
        }
      }
    }
  }
  double* outp = a.Pp + (int64_t)blockIdx.x * k2 * r;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ai = ta + 16 * i, c = tb + 16 * j;
      if (ai < k2 && c < r) outp[ai * r + c] = acc[i][j];
    }
}

template <typename T>
hipError_t launch_nmf_row(const RowArgs& a0, int blocks, hipStream_t st) {
  RowArgs a = a0;
  if (a.r > 64 || (a.B2 && a.k2 > 128) || (a.C && a.k1 > 128)) return hipErrorInvalidValue;
  a.rows_per_block = (a.rows + blocks - 1) / blocks;
  const int k2 = a.B2 ? a.k2 : a.r;
  size_t sm = ((a.C ? (size_t)a.k1 * a.r : 0) + 2 * (size_t)a.r * a.r + 3 * (size_t)kRowCh * (a.r + 1) +
               (size_t)kRowCh * (k2 + 1)) * sizeof(double);
  if ((size_t)kRowCh * ((a.r + 3) / 4) > 256) return hipErrorInvalidValue;
  if (sm > 160 * 1024) return hipErrorInvalidValue;
  hipFuncSetAttribute((const void*)nmf_row_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  hipLaunchKernelGGL(nmf_row_kernel<T>, dim3(blocks), dim3(256), sm, st, a);
  CNMF_LAUNCH_CHECK();
}
template hipError_t launch_nmf_row<float>(const RowArgs&, int, hipStream_t);
template hipError_t launch_nmf_row<double>(const RowArgs&, int, hipStream_t);

// ---------------------------------------------------------------------------
// Small step between half-steps (one workgroup, after the fixed-order
// reduction of the partials into S):
//   MU, C form:    C = S (k x r), G = C^T C, G+ = max(G, 0), G- = max(-G, 0)
//   MU, Gram form: G = S (r x r), G+, G-
//   ANLS, C form:  G = C^T C (C = S, k x r), unsplit
// ((Gram + pen I)^-1 of the uncompressed ADMM: launch_spd_inverse below)
// ---------------------------------------------------------------------------
constexpr int kSmallNT = 256;

__global__ __launch_bounds__(kSmallNT) void nmf_small_kernel(const double* __restrict__ S, int k, int r, int mode,
                                                             double pen, double* __restrict__ Gp,
                                                             double* __restrict__ Gm, int* flags) {
  // S (k x r, k <= 128, r <= 64) staged in LDS first, with eight loads in
  // flight per thread; the products then read LDS in the same order as before
  __shared__ double Ss[128 * 64];
  const int tid = threadIdx.x;
  const int cnt = mode == 1 ? r * r : k * r;
  staged_copy<8>(cnt, tid, kSmallNT, [&](int e) { return S[e]; }, [&](int e, double v) { Ss[e] = v; });
  __syncthreads();
  if (mode == 3) {
    for (int e = tid; e < r * r; e += kSmallNT) {
      const int a = e / r, b = e - a * r;
      double s0 = 0.0, s1 = 0.0;
      int l = 0;
      for (; l + 1 < k; l += 2) {
        s0 = fma(Ss[l * r + a], Ss[l * r + b], s0);
        s1 = fma(Ss[(l + 1) * r + a], Ss[(l + 1) * r + b], s1);
      }
      if (l < k) s0 = fma(Ss[l * r + a], Ss[l * r + b], s0);
      Gp[e] = s0 + s1;
    }
    return;
  }
  if (mode == 0 || mode == 1) {
    for (int e = tid; e < r * r; e += kSmallNT) {
      const int a = e / r, b = e - a * r;
      double g;
      if (mode == 0) {
        double s0 = 0.0, s1 = 0.0;
        int l = 0;
        for (; l + 1 < k; l += 2) {
          s0 = fma(Ss[l * r + a], Ss[l * r + b], s0);
          s1 = fma(Ss[(l + 1) * r + a], Ss[(l + 1) * r + b], s1);
        }
        if (l < k) s0 = fma(Ss[l * r + a], Ss[l * r + b], s0);
        g = s0 + s1;
      } else {
        g = Ss[e];
      }
      Gp[e] = g > 0.0 ? g : 0.0;
      Gm[e] = g < 0.0 ? -g : 0.0;
    }
    return;
  }
}


hipError_t launch_nmf_small(const double* S, int k, int r, int mode, double pen, double* Gp, double* Gm, int* flags,
                            hipStream_t st) {
  if (mode < 0 || mode > 3 || mode == 2 || r < 1 || r > 64 || (mode != 1 && (k < 1 || k > 128)))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(nmf_small_kernel, dim3(1), dim3(kSmallNT), 0, st, S, k, r, mode, pen, Gp, Gm, flags);
  CNMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// (S + pen I)^-1 through the one-wave Cholesky of the orthonormalisation:
// G = sym(S) + pen I, G = T^T T, Minv = T^-1 T^-T (T^-1 upper triangular),
// optionally checked against G.
// ---------------------------------------------------------------------------
__global__ void spd_prep_kernel(const double* __restrict__ S, int r, double pen, double* __restrict__ G,
                                int* __restrict__ floored) {
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int i = e / r, j = e - i * r;
    G[e] = 0.5 * (S[i * r + j] + S[j * r + i]) + (i == j ? pen : 0.0);
  }
  if (threadIdx.x == 0) *floored = 0;
}

__global__ __launch_bounds__(256) void spd_inv_finish_kernel(const double* __restrict__ G,
                                                             const double* __restrict__ Ti, int r,
                                                             double* __restrict__ Minv,
                                                             const int* __restrict__ floored, int* ok) {
  __shared__ double Ms[64 * 65];
  __shared__ double Ts[64 * 64];   // Ti, then G (both r x r, r <= 64)
  __shared__ double worst[256];
  const int tid = threadIdx.x;
  // operands staged in LDS with eight loads in flight per thread; the sums
  // read them in the same order as from global memory
  staged_copy<8>(r * r, tid, 256, [&](int e) { return Ti[e]; }, [&](int e, double v) { Ts[e] = v; });
  __syncthreads();
  for (int e = tid; e < r * r; e += 256) {
    const int i = e / r, j = e - i * r;
    double s = 0.0;
    for (int l = max(i, j); l < r; ++l) s = fma(Ts[i * r + l], Ts[j * r + l], s);
    Ms[i * 65 + j] = s;
    Minv[e] = s;
  }
  if (!ok) return;
  __syncthreads();
  staged_copy<8>(r * r, tid, 256, [&](int e) { return G[e]; }, [&](int e, double v) { Ts[e] = v; });
  __syncthreads();
  double err = 0.0;
  for (int e = tid; e < r * r; e += 256) {
    const int i = e / r, j = e - i * r;
    double s = (i == j) ? -1.0 : 0.0;
    for (int l = 0; l < r; ++l) s = fma(Ts[i * r + l], Ms[l * 65 + j], s);
    err = (s == s) ? fmax(err, fabs(s)) : INFINITY;
  }
  worst[tid] = err;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) worst[tid] = fmax(worst[tid], worst[tid + w]);
    __syncthreads();
  }
  if (tid == 0) *ok = (worst[0] <= 1e-8 && *floored == 0) ? 1 : 0;
}

hipError_t launch_spd_inverse(const double* S, int r, double pen, double* G, double* Tinv, double* Minv, int* floored,
                              int* ok, hipStream_t st) {
  if (r < 1 || r > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(spd_prep_kernel, dim3(1), dim3(256), 0, st, S, r, pen, G, floored);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  CholOpts o{};
  o.tau = 1e-300;
  o.unresolved = floored;
  e = launch_chol_tinv(G, 1, r, Tinv, o, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spd_inv_finish_kernel, dim3(1), dim3(256), 0, st, G, Tinv, r, Minv, floored, ok);
  CNMF_LAUNCH_CHECK();
}

}  // namespace cnmf
