"""CPU FP64 reference (test infrastructure only; never on the product path).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.
"""
from .oracle import (  # noqa: F401
    OracleError,
    build,
    diag,
    expect_pauli,
    library_path,
    max_threads,
    run,
    run_on,
    sample_block,
    statevector,
    trace_distance,
    vec_to_matrix,
    matrix_to_vec,
    readout_probs,
    sample,
    splitmix64,
    reduced_dm,
    process_chi_1q,
)
