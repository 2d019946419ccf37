"""The persistent projection and OC kernels launched plainly (the default:
a grid that fits the device at once) and through the runtime's cooperative
launch give bit-identical results: the same kernels, the same block count,
the same fixed-order reductions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05436_amd import _lib
    _lib.load()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("precision,ft", [("f64", 3), ("f32", 1), ("f32", 2)])
def test_plain_and_cooperative_launches_agree(precision, ft):
    from dataclasses import replace
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    cfg = replace(W.C1[300], iterations=5, precision=precision, ft=ft)
    a = TopOpt(cfg, autotune=False)
    b = TopOpt(cfg, autotune=False)
    assert L.to_plan_get_tuning(a.plan.handle).coop_launch == 0
    L.to_plan_set_tuning(b.plan.handle, 8, 0, 256, 0, coop_launch=1)
    assert L.to_plan_get_tuning(b.plan.handle).coop_launch == 1
    for k in range(5):
        a.step()
        b.step()
        assert np.array_equal(host(a.x), host(b.x)), k
        assert np.array_equal(host(a.xphys), host(b.xphys)), k
        sa, sb = a.stats(), b.stats()
        assert sa["n_bs"] == sb["n_bs"] and sa["lmid"] == sb["lmid"], k
    with pytest.raises(L.ToError):
        L.to_plan_set_tuning(b.plan.handle, 8, 0, 256, 0, coop_launch=2)
