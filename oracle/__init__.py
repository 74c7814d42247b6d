"""Plain FP64 CPU oracle for the cosine-transform t-SVD / t-SVT hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_1902_03070_amd``) never imports it, and the two share no code.
"""
from .oracle import (  # noqa: F401
    build,
    set_threads,
    host_threads,
    dct_matrix,
    dct_tubes,
    idct_tubes,
    split_shift,
    bt,
    bh,
    btph,
    unfold,
    fold,
    btph_product,
    tprod_dct,
    jacobi_svd,
    tsvd_dct,
    tsvd_dct_full,
    tsvt_dct,
    tnn_c,
    complete,
    tsvt_transform,
    dft_tubes,
    idft_tubes,
    bcirc,
    svt_complex,
    tsvt_dft,
    tnn_f,
)
