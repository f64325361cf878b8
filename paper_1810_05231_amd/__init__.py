"""MI355X (gfx950) implementation of the low-rank PDHG method for general SDPs
(Souto, Garcia, Veiga, arXiv 1810.05231): PD-SDP (Algorithm 1) and LR-PD-SDP
(Algorithm 2) with the truncated PSD projection of Section 3.1, as the HIP
library libproxsdp.so behind the C interface of include/proxsdp.h.
"""
from ._lib import FP32, FP64, BF16, ProxSDPError, lib  # noqa: F401
from .solver import Solver, project_psd, project_psd_noalloc, workspace_size  # noqa: F401

__all__ = ["Solver", "project_psd", "project_psd_noalloc", "workspace_size", "ProxSDPError", "lib"]
