"""Pin of the byte accounting used for the roofline: one read and one write
of every population per site and step (Section 4 notes that non-temporal
stores remove the write-allocate read). Table 1 of the paper converts its
propagate times to GB/s with exactly this count."""
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_propagate.txt")


def _rows():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, t_ms, gbs = line.split()
        lattice = (4608, 12288) if "4608x12288" in name else (1024, 8192)
        out.append((name, lattice, float(t_ms), float(gbs)))
    return out


@pytest.mark.parametrize("row", _rows(), ids=lambda r: r[0])
def test_table1_bandwidth_from_two_transfers_per_population(row):
    from paper_1804_01918_amd.roofline import bytes_per_site
    _, (lx, ly), t_ms, gbs = row
    got = bytes_per_site("f64", fused=True) * lx * ly / (t_ms * 1e-3) / 1e9
    assert abs(got / gbs - 1) < 0.06


def test_table1_footprint():
    """About 4.6 GB for 1024 x 8192: two copies of 37 doubles per site."""
    from paper_1804_01918_amd.roofline import bytes_per_site
    gib = 1024 * 8192 * bytes_per_site("f64", fused=True) / 2**30
    assert abs(gib - 4.625) < 1e-9
