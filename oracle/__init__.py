"""CPU FP64 oracle for the fermion determinant -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct numpy/scipy implementations of what the GPU
path computes.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library never does.  It shares no code
with the HIP path.
"""
from .fdet_oracle import (  # noqa: F401
    slice_exponential,
    slice_matrices,
    block_fermion_matrix,
    block_matrix_of_slices,
    bruteforce_logdet_greens,
    bruteforce_force,
    dense_logdet_greens,
    stabilised_logdet_greens,
    sporadic_logdet_greens,
    dsplit_logdet_greens,
    stabilised_force,
    stabilised_force_rows,
    udv_identity,
    udv_product,
    udv_close,
    wrap_phase,
    logdet_close,
    response_trace,
    diag_response,
    slice_response,
    displaced_split,
    bruteforce_displaced_greens,
    displaced_greens,
    dsplit_displaced_greens,
    taylor_product_coefficients,
    taylor_slice_matrices,
    sparse_logdet_greens,
    hmc_hamiltonian,
    hmc_leapfrog,
)
from .closed_form import (  # noqa: F401
    honeycomb_dispersion,
    uniform_field_logdet,
    uniform_field_greens,
    uniform_field_force,
    uniform_field_displaced_greens,
    uniform_field_taylor_logdet_greens,
    two_site,
    two_site_displaced,
    two_site_taylor,
    two_site_slice_response,
)
