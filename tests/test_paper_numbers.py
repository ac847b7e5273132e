"""The paper's printed throughput and bandwidth figures (Table 1, Table 2 and the
text of Section 2.1), reproduced by the byte model bench.py uses to quote them as
context.  Values are stored in tests/golden with their citation."""
import os

import numpy as np

import bench

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_table1_bandwidth_model():
    for r in _rows("paper_table1.txt"):
        dim, mhz = int(r[0]), float(r[1])
        fp_bits, idx_bits = bench.paper_bits_per_point(dim)
        assert (fp_bits, idx_bits) == (int(r[2]), int(r[3]))
        gfp, gidx = bench.paper_required_gbps(dim, mhz)
        assert abs(gfp - float(r[4])) < 0.05 and abs(gidx - float(r[5])) < 0.05
        gfp3, gidx3 = bench.paper_required_gbps(dim, 300)
        assert abs(gfp3 - float(r[6])) < 0.05 and abs(gidx3 - float(r[7])) < 0.05
        # naive port: one memory read per cycle over (values + indices) / 4 banks...
        # the printed points/cycle times the clock gives the printed Mpoints/s
        assert abs(float(r[9]) * mhz - float(r[10])) / float(r[10]) < 0.01
        # II = 1 core: one point per cycle, so FLOP/point = GFLOPS / clock
        flop_per_point = float(r[8]) * 1e9 / (mhz * 1e6)
        assert 40 < flop_per_point < 200


def test_table2_percentages():
    desired = np.array([56.0, 60.0, 33.6, 50.4])   # Table 1: fp + index GB/s
    errata = []
    for r in _rows("paper_table2.txt"):
        pct = np.array([float(v) for v in r[2:]])
        computed = 100.0 * float(r[1]) / desired
        bad = np.abs(computed - pct) > np.maximum(1.0, 0.002 * pct)   # printed rounding (821.4 -> 820)
        errata += [(r[0], i) for i in np.nonzero(bad)[0]]
    # the one printed cell that does not follow from its row: 1 channel
    # DDR4-2666 at 300 MHz in 3D (printed 59%, 21.3/50.4 = 42%)
    assert errata == [("ddr4_2666_1ch", 3)]
