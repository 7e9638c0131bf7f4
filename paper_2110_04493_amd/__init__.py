"""MI355X (gfx950) filtered precise-integration sparse matrix exponential.

Submodules: ``capi`` (ctypes binding of include/expm.h), ``api`` (torch
tensors in and out), ``workloads`` (seeded synthetic inputs), ``build``
(compiles the HIP library).  Importing the package loads nothing; the HIP
library is loaded on first use and its absence raises.
"""
__all__ = ["capi", "api", "workloads", "build"]
