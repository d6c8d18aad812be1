"""MI355X-native compressed NMF (Tepper & Sapiro, arXiv:1505.04650).

The compute path is the HIP library libcnmf.so (C ABI in include/cnmf.h);
``paper_1505_04650_amd.api`` is its Python binding.  Importing the package
does not load the library; the binding loads it on first use and raises if
it has not been built.
"""

__all__ = ["api", "workloads"]
