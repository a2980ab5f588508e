"""MI355X-native hot path of convolutional-RBM-aided Monte Carlo
(Alcalde Puente & Eremin, arXiv:2008.05401).

Submodules:
  _lib       ctypes binding of libcrbm.so (the C ABI of include/crbm.h)
  api        torch-facing wrappers (device memory and streams only)
  workloads  seeded synthetic inputs (filters, temperatures, job streams)
  serve      continuous-batching job server
  build      hipcc build of libcrbm.so
"""

__all__ = ["api", "workloads", "build"]
