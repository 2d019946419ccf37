"""The whole redesign loop on the GPU against compliance values the paper
prints.  Fig. 7 (Sec. 4): the 3D cantilever 48 x 24 x 24, volume fraction
0.12, rmin sqrt(3), volume-preserving projection, after 100 redesign steps:
c = 3993.7 with the zero-Neumann filter boundary rule and 4074.3 with the
zero-Dirichlet one.  The paper's code and this library take different
rounding paths through 100 nonlinear steps (and the run's beta and move
limit are the code's defaults, 2 and 0.2), so the bar is 3%; the runs here
land within 2%."""
from dataclasses import replace

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


@pytest.mark.parametrize("bc,paper_c", [("N", 3993.7), ("D", 4074.3)])
def test_cantilever3d_48_compliance_after_100_steps(bc, paper_c):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    cfg = replace(W.C2, name="cantilever48x24x24", nelx=48, nely=24, nelz=24, bc=bc, iterations=100)
    g = TopOpt(cfg, precond=L.TO_PREC_GMG)
    for _ in range(100):
        g.step()
    s = g.stats()
    assert s["solve_ok"] and s["newton_ok"] and abs(s["vol"] - 0.12) <= 1e-6
    assert abs(s["c"] - paper_c) <= 0.03 * paper_c, (bc, s["c"], paper_c)
    print(f"3D cantilever 48x24x24 '{bc}': c = {s['c']:.1f} after 100 steps (paper {paper_c})")
