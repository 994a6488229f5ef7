"""MI355X (gfx950) preconditioned Landweber deblurring under Anti-Reflective
boundary conditions: Python binding of the HIP library libardeblur.so.

The binding only marshals arguments; every step of the method runs in the
library's HIP kernels.  Build the library with
``python -m paper_1211_0393_amd.build``."""

from ._lib import (  # noqa: F401
    AR_ADJOINT,
    AR_BC_ANTIREFLECTIVE,
    AR_BC_PERIODIC,
    AR_BC_REFLECTIVE,
    BCS,
    AR_F32,
    AR_F32_ACC64,
    AR_F32_BF16X3,
    AR_F64,
    DTYPES,
    AR_FILTER_GAINS,
    AR_FILTER_IDENTITY,
    AR_FNET_BINS,
    AR_FNET_IN,
    AR_FNET_NPARAM,
    AR_FILTER_THRESHOLD,
    AR_FILTER_TIKHONOV,
    AR_REBLUR,
    AR_TUNE_BLUR,
    AR_TUNE_FUSE,
    AR_TUNE_COL_ALGO,
    AR_TUNE_COL_EXCL,
    AR_TUNE_COL_LANES,
    AR_TUNE_COL_WAVES,
    AR_TUNE_ROW_ALGO,
    AR_TUNE_ROW_EXCL,
    AR_TUNE_ROW_LANES,
    AR_TUNE_ROW_WAVES,
    ArError,
    Batch,
    FNet,
    LIB_PATH,
    Plan,
    SIGNATURES,
    ar_psf_normalize,
    load,
    version,
)
