"""Seeded synthetic inputs (Philox4x32-10 counters) shared by the oracle and
the GPU path.  Input generation only: no polarization arithmetic lives here."""
from .philox import philox4x32
from .workloads import (Block, Workload, workload, z_scale_table, vsqrt_table, hist_edges,
                        gauss_legendre_imag_axis, c3_word, KEY0, KEY1, TAG_Z, TAG_WC)

__all__ = ["philox4x32", "Block", "Workload", "workload", "z_scale_table", "hist_edges",
           "vsqrt_table", "gauss_legendre_imag_axis", "c3_word", "KEY0", "KEY1",
           "TAG_Z", "TAG_WC"]
