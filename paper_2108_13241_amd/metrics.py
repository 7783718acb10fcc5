"""Performance metrics of the lattice-Boltzmann step (pure arithmetic, no GPU).

Sec. 4.3 of the paper defines performance in lattice updates per second (LUPS); since the
method is bandwidth-bound it also expresses it as the minimal bandwidth that rate needs:
B_node = 2 q s_d bytes per node (read and write every population once), P_B = B_node * LUPS
and U_B = P_B / B_peak.  Only non-solid nodes count (Eq. 8's porosity is their fraction).
The measurements here additionally count the 1-byte node type per node (18 s_d + 1), and 4
bytes per node of drag coefficient when a drag field is present.
"""
from __future__ import annotations

POP_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
MI355X_HBM_PEAK_GBPS = 8000.0  # AMD public specification (HBM3E)


def glups(fluid_nodes: int, steps: int, seconds: float) -> float:
    return fluid_nodes * steps / seconds / 1e9


def paper_bytes_per_node(s_d: int, q: int = 9) -> int:
    """B_node = 2 q s_d (Sec. 4.3)."""
    return 2 * q * s_d


def bytes_per_node(dtype: str, drag: bool = False) -> int:
    """18 populations moved (read + write) + the node-type byte [+ 4 B drag field]."""
    return 18 * POP_BYTES[dtype] + 1 + (4 if drag else 0)


def bandwidth_gbps(glups_value: float, node_bytes: float) -> float:
    """P_B in GB/s for a rate in GLUPS."""
    return glups_value * node_bytes


def utilisation(gbps: float, peak_gbps: float) -> float:
    """U_B = P_B / B_peak."""
    return gbps / peak_gbps


def porosity(n_non_solid: int, n_all: int) -> float:
    """phi of Eq. 8: the fraction of non-solid nodes."""
    return n_non_solid / n_all


def sparse_efficiency(p_sparse: float, p_dense: float) -> float:
    """eta_P of Eq. 9: performance on a sparse geometry over performance on the dense one,
    same data layout and geometry size (performance counts non-solid nodes only)."""
    return p_sparse / p_dense
