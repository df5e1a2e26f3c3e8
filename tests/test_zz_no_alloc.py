"""The statistics entry point that allocates nothing (lbm_stats_noalloc), called through the C
ABI, against lbm_residual on identical runs: two calls in a row on a larger run, then one on a
smaller run (fewer statistics blocks share the same device scratch array)."""
import numpy as np
import pytest

from paper_2606_29619_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
capi = pytest.importorskip("paper_2606_29619_amd.capi")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    capi.load()
    yield
    torch.cuda.synchronize()


def _pair(shape, storage, seed):
    w = workloads.random_porosity_3d(shape=shape, seed=seed, ell=3.0, nu=0.03, b=2e-4)
    m = np.zeros(shape, np.uint8)
    m[1:3, 2:4, 3:6] = 1
    w.mask = m
    return (capi.Solver.from_workload(w, storage=storage),
            capi.Solver.from_workload(w, storage=storage))


def _check(a, b, steps):
    """lbm_residual on a, lbm_stats_noalloc on b (same run, same steps): all eight slots equal
    bit for bit."""
    a.step(steps)
    b.step(steps)
    ra = a.residual()
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    capi.lbm_stats_noalloc(b.handle, out.data_ptr())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.array([ra.mass, ra.momentum[0], ra.momentum[1], ra.momentum[2], ra.vmax, ra.dv2,
                     ra.v2, float(ra.nonfinite)])
    print("noalloc stats", got.tolist(), flush=True)
    assert np.array_equal(got, want), (got, want)
    return got


def test_stats_noalloc_matches_lbm_residual():
    a, b = _pair((40, 48, 64), capi.LBM_F32, 3)        # 480 statistics blocks
    first = _check(a, b, 5)
    assert first[6] == 0.0                              # no earlier snapshot
    second = _check(a, b, 6)                            # residual against the first call
    assert second[5] > 0 and second[6] > 0
    c, d = _pair((6, 9, 10), capi.LBM_F64, 4)           # 3 blocks: a smaller input
    _check(c, d, 7)
    _check(c, d, 2)
    for s in (a, b, c, d):
        s.close()


def test_stats_noalloc_rejects_bad_arguments():
    a, _ = _pair((4, 5, 6), capi.LBM_F32, 5)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_stats_noalloc(a.handle, 0)
    assert ei.value.code == capi.LBM_ERR_INVALID_ARG
    a.close()
