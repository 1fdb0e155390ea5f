"""CPU oracle for the rank-1 SVD update -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It shares no code with the HIP path.
"""
from .svdu_oracle import (  # noqa: F401
    gram_split, deflate, secular_roots, secular_f, loewner_weights, rank_one_update, rank_one_update_z,
    svd_rank1_update, svd_rankk_update, dense_ahat, recon_error, paper_error, orth_error, U64,
)
from .jacobi import jacobi_svd  # noqa: F401
