"""ka_footprint (the figure the job server admits by) against the device memory a sim really
takes: after an init, sweeps on either path and a ka_run with observations, the device's free
memory has dropped by no more than the footprint, the ka_run's count buffers and the
allocation granularity; freeing the sim returns it."""
import pytest
import torch

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu

SLACK = 32 << 20   # allocation granularity over a sim's dozen device buffers


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


@pytest.fixture(scope="module", autouse=True)
def warm():
    # load the library's code objects and the runtime's own buffers before measuring
    for path in (1, 2):
        g = ka.ka_graph_lattice(2, 8)
        s = ka.ka_init(g, 2, 0.5, 1, 64)
        ka.ka_set_option(s, ka.KA_OPT_PATH, path)
        ka.ka_sweep(s, 2)
        ka.ka_run(s, [3, 4])
        s.free()
    yield


@pytest.mark.parametrize("kind,args,R,path", [
    ("lat", (3, 128), 256, 1),
    ("lat", (2, 64), 64, 2),
    ("lat", (3, 16), 128, 2),
    ("rrg", (1 << 18, 4, 5), 64, 1),
    ("rrg", (2000, 4, 5), 64, 2),
])
def test_footprint_bounds_device_memory(kind, args, R, path):
    _say(f"footprint {kind} {args} R={R} path={path}")
    g = ka.ka_graph_lattice(*args) if kind == "lat" else ka.ka_graph_rrg(*args)
    fp = ka.ka_footprint(g, R)
    before = _free_bytes()
    s = ka.ka_init(g, 2, 0.7, 3, R)
    ka.ka_set_option(s, ka.KA_OPT_PATH, path)
    ka.ka_sweep(s, 3)
    times = [4, 5, 8]
    ka.ka_run(s, times)
    ka.ka_observe(s)
    used = before - _free_bytes()
    run_bytes = len(times) * 3 * R * 8 + len(times) * 8   # ka_run's counts and times
    assert used <= fp + run_bytes + SLACK, (used, fp)
    if kind == "lat" and args == (3, 128):
        # the three state arrays dominate: the footprint is not padded far beyond them
        assert used >= 0.9 * fp, (used, fp)
    s.free()
    assert before - _free_bytes() <= SLACK
