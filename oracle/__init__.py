"""CPU FP64 oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything under ``oracle/``.  It shares no code with the
GPU library; its inputs come from the seeded generator in ``synth/``.
"""
from .chi0_oracle import *  # noqa: F401,F403
from .chi0_oracle import (chi0_ref, chi0_brute, chi0_exact, chi0_entries, chi0_rows,
                          chi0_block, chi0_workload, dielectric, inverse,
                          inverse_gauss_jordan, screened_wc, transition_weight,
                          pair_delta, pair_included, rel_fro, workload_blocks)
from .sigx_oracle import sigx_block, sigx_brute, sigx_exact, sigx_ref  # noqa: F401
from .sigc_oracle import (ag_weights, ag_weight_table, sigc_block, sigc_brute,  # noqa: F401
                          sigc_contract, sigc_contract_exact, sigc_entries, sigc_ref,
                          sigc_rows)
from .hist_oracle import (bin_fractions, hilbert_apply, hilbert_imag, hilbert_real,  # noqa: F401
                          hist_brute, hist_entries, hist_exact, hist_ref, log_edges)
