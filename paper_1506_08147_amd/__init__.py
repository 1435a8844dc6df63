"""MI355X library for DGDFT's adaptive-local-basis generation (Hu, Lin, Yang,
Sec. II.A-B): batched planewave local eigenproblems solved by Teter-
preconditioned LOBPCG in hand-written HIP kernels, then restriction to the
element and SVD truncation to ALBs.

This package is a thin ctypes binding over the C ABI in include/dgdft_alb.h
(libdgdft_alb.so, built in-tree).  It marshals arguments only; every step of
the method runs in the library's kernels.  It raises if the library is not
built: there is no CPU fallback.
"""
from .binding import (  # noqa: F401
    ALB,
    LibraryMissing,
    DGDFTError,
    gemm_batched,
    load_library,
    mlp_eval,
    mlp_grad,
    mlp_train,
    small_gemm_batched,
    small_syev,
    small_syev_noalloc,
    LIB_PATH,
    EXPORTS,
)
