"""ka_observe_noalloc (the observation entry point for callers that cannot allocate device
memory) through the C ABI: its counts equal ka_observe's on two calls in a row, the second on
a smaller sim (fewer replicas, so the shared scratch still holds the first call's larger
contents), it leaves the device's free memory unchanged, and it rejects more replicas than
its fixed scratch holds."""
import ctypes

import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _free_device_bytes():
    """hipMemGetInfo of the current device, from the HIP runtime libka itself uses."""
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipDeviceSynchronize() == 0
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def test_noalloc_observe_equals_observe():
    big = ka.ka_init(ka.ka_graph_lattice(3, 16), 3, 0.7, 4, 256)       # 3 x 256 counts
    small = ka.ka_init(ka.ka_graph_rrg(500, 4, 8), 2, 0.6, 5, 64)        # 3 x 64 counts
    ka.ka_sweep(big, 7)
    ka.ka_sweep(small, 4)
    _say("noalloc observe: 3D L=16 x 256 replicas, then RRG N=500 x 64 replicas")
    first = ka.ka_observe_noalloc(big)
    before = _free_device_bytes()
    second = ka.ka_observe_noalloc(small)
    after = _free_device_bytes()
    assert before == after, "ka_observe_noalloc changed the free device memory"
    for sim, got in ((big, first), (small, second)):
        want = ka.ka_observe(sim)
        assert got[0] == want[0]
        for a, b in zip(got[1:], want[1:]):
            assert np.array_equal(a, b)
    # and again after more sweeps, small then big
    ka.ka_sweep(small, 3)
    ka.ka_sweep(big, 2)
    for sim in (small, big):
        got = ka.ka_observe_noalloc(sim)
        want = ka.ka_observe(sim)
        assert got[0] == want[0] == sim.t
        for a, b in zip(got[1:], want[1:]):
            assert np.array_equal(a, b)
    big.free()
    small.free()


def test_noalloc_observe_rejects_too_many_replicas():
    sim = ka.ka_init(ka.ka_graph_lattice(2, 4), 2, 0.5, 1, 8192 + 64)
    _say("noalloc observe: 8256 replicas rejected")
    with pytest.raises(ka.KaError) as e:
        ka.ka_observe_noalloc(sim)
    assert e.value.code == ka.KA_EINVAL
    n_t = ctypes.c_int64()
    assert ka.load().ka_observe_noalloc(sim.handle, ctypes.byref(n_t), None, None, None) == ka.KA_EINVAL
    sim.free()
