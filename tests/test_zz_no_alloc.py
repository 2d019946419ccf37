"""to_sensitivity_noalloc (the allocation-free variant of to_sensitivity,
whose compliance-sum scratch is a static device array of the library)
against to_sensitivity, through the C ABI: element sensitivities of eq. (7)
and the compliance f.u bit-identical, on two calls in a row, the second on a
smaller mesh; also a repeat of the first call after the smaller one (the
shared scratch keeps the last call's contents)."""
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


def _case(dims, dt, seed):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan
    dim = len(dims)
    nelx, nely = dims[0], dims[1]
    nelz = dims[2] if dim == 3 else 1
    # clamp the x = 0 face (any supports will do for this comparison)
    nn = (nely + 1) * ((nelz + 1) if dim == 3 else 1)
    fixed = np.arange(dim * nn, dtype=np.int32)
    m = nelx * nely * nelz
    passive = np.zeros(m, np.uint8)
    passive[::13] = L.TO_SOLID
    passive[5::29] = L.TO_VOID
    P = Plan(dim, nelx, nely, nelz, rmin=1.5, bc="D", fixed=fixed, passive=passive)
    n = P.info.n
    T = torch.float64 if dt == L.TO_F64 else torch.float32
    x = torch.as_tensor(W.design_field(m, seed), dtype=T).cuda()
    u = torch.as_tensor(W.displacement_field(n, seed + 1), dtype=torch.float64).cuda()
    f = torch.as_tensor(W.displacement_field(n, seed + 2), dtype=torch.float64).cuda()
    return P, x, u, f


def _both(P, dt, x, u, f, penal):
    from paper_2005_05436_amd import _lib as L
    m = P.info.m
    T = x.dtype
    dc_a = torch.full((m,), 7.0, dtype=T, device="cuda")
    dc_b = torch.full((m,), -7.0, dtype=T, device="cuda")
    c_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    c_b = torch.full((1,), 123.0, dtype=torch.float64, device="cuda")
    L.to_sensitivity(P.handle, dt, x, u, f, penal, dc_a, c_a)
    L.to_sensitivity_noalloc(P.handle, dt, x, u, f, penal, dc_b, c_b)
    torch.cuda.synchronize()
    return dc_a.cpu().numpy(), dc_b.cpu().numpy(), c_a.item(), c_b.item()


@pytest.mark.parametrize("dt", [1, 0])
@pytest.mark.parametrize("big,small", [((400, 200), (30, 10)), ((40, 20, 20), (6, 4, 3))])
def test_noalloc_matches_to_sensitivity(big, small, dt):
    print(f"no-alloc sensitivity: dtype {dt}, meshes {big} then {small} then {big}", flush=True)
    P1, x1, u1, f1 = _case(big, dt, 31)
    P2, x2, u2, f2 = _case(small, dt, 41)
    for P, x, u, f, penal in ((P1, x1, u1, f1, 3.0), (P2, x2, u2, f2, 2.5), (P1, x1, u1, f1, 3.0)):
        a, b, ca, cb = _both(P, dt, x, u, f, penal)
        np.testing.assert_array_equal(a, b)
        assert ca == cb, (ca, cb)
        ref = float(f.cpu().numpy() @ u.cpu().numpy())
        assert abs(cb - ref) <= 1e-12 * np.abs(f.cpu().numpy()).sum() * np.abs(u.cpu().numpy()).max()
    # without the compliance sum (f = NULL): element values only
    m = P2.info.m
    dc_a = torch.zeros(m, dtype=x2.dtype, device="cuda")
    dc_b = torch.ones(m, dtype=x2.dtype, device="cuda")
    from paper_2005_05436_amd import _lib as L
    L.to_sensitivity(P2.handle, dt, x2, u2, None, 3.0, dc_a, None)
    L.to_sensitivity_noalloc(P2.handle, dt, x2, u2, None, 3.0, dc_b, None)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dc_a.cpu().numpy(), dc_b.cpu().numpy())
    P1.close()
    P2.close()


def test_noalloc_rejects_bad_arguments():
    from paper_2005_05436_amd import _lib as L
    P, x, u, f = _case((30, 10), 1, 51)
    dc = torch.zeros(P.info.m, dtype=torch.float64, device="cuda")
    with pytest.raises(L.ToError):
        L.to_sensitivity_noalloc(P.handle, 1, x, None, f, 3.0, dc, None)
    with pytest.raises(L.ToError):
        L.to_sensitivity_noalloc(P.handle, 7, x, u, f, 3.0, dc, None)
    P.close()
