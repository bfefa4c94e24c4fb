"""The dependent-load latency probe: a trip that misses the L2 takes longer than one that
hits it, and every figure is finite and within what a memory trip can take."""
import pytest

import paper_2408_09399_amd as tm

pytestmark = pytest.mark.gpu


def test_latency_probe_orders_l2_and_hbm():
    l2_1 = tm.load_latency_ns(1 << 20, lanes=1, steps=4000)
    l2_64 = tm.load_latency_ns(1 << 20, lanes=64, steps=4000)
    hbm_1 = tm.load_latency_ns(4 << 30, lanes=1, steps=4000)
    hbm_64 = tm.load_latency_ns(4 << 30, lanes=64, steps=4000)
    print(f"ns per trip: L2 {l2_1:.0f} / {l2_64:.0f} (1 / 64 lines), HBM {hbm_1:.0f} / {hbm_64:.0f}", flush=True)
    for v in (l2_1, l2_64, hbm_1, hbm_64):
        assert 20.0 < v < 20000.0
    assert hbm_1 > l2_1 and hbm_64 > l2_64
