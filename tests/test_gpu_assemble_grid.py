"""The assembly kernels (the segmented sum over the permutation of I_r, one
thread per slot with the slot's row from row_ptr and its contributing
elements from the grid, and in 2D one thread per node writing its two rows)
give bit-identical values: the same terms in the same order (ascending pair
index t), on meshes with ragged tiles and at the benchmark's size.  Also against the oracle's segmented
sum, and the tuning's validation of the kernel choice."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W
from oracle import element as oel
from oracle import mesh as omesh
from oracle import sparse as osp


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05436_amd import _lib
    _lib.load()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _plan(dims):
    from paper_2005_05436_amd.driver import Plan
    nelz = dims[2] if len(dims) == 3 else 1
    return Plan(len(dims), dims[0], dims[1], nelz, 2.0, "D", (), None)


@pytest.mark.parametrize("dt", [1, 0])   # TO_F64, TO_F32
@pytest.mark.parametrize("dims", [(6, 4), (60, 20), (37, 21), (1200, 400), (6, 4, 3), (6, 5, 4), (8, 7, 5),
                                  (96, 48, 48)])
def test_grid_kernel_matches_segmented_kernel(dims, dt):
    from paper_2005_05436_amd import _lib as L
    P = _plan(dims)
    M = omesh.Mesh(*dims)
    T = torch.float64 if dt == L.TO_F64 else torch.float32
    x = W.design_field(M.m, 21)
    x[: min(5, M.m)] = 0.0
    xd = torch.as_tensor(x, dtype=T).cuda()
    out = {}
    for rows in ((0, 1, 2) if len(dims) == 2 else (0, 1)):
        for nt in (128, 256, 512):
            L.to_plan_set_tuning(P.handle, 8, 0, nt, 0, asm_rows=rows)
            assert L.to_plan_get_tuning(P.handle).asm_rows == rows
            kval = torch.full((P.info.nnz_lower,), float("nan"), dtype=T, device="cuda")
            L.to_assemble(P.handle, dt, xd, 3.0, kval)
            out[rows, nt] = host(kval)
    ref = out[0, 256]
    assert not np.isnan(ref).any()
    for k, v in out.items():
        np.testing.assert_array_equal(v, ref, err_msg=str(k))
    if M.m <= 20000:
        ke = oel.element_matrix(M.dim, 0.3)
        _, _, perm, seg_ptr = osp.csr_pattern(osp.reduced_index_set(M.cmat()), M.n)
        want = osp.assemble(host(xd).astype(np.float64), oel.lower_vector(ke), perm, seg_ptr, 3.0, 1.0, 1e-9)
        err = np.abs(out[1, 256] - want).max() / np.abs(want).max()
        assert err < (1e-13 if dt == L.TO_F64 else 1e-6)


def test_grid_kernel_choice_is_validated():
    from paper_2005_05436_amd import _lib as L
    P = _plan((6, 4))
    with pytest.raises(L.ToError):
        L.to_plan_set_tuning(P.handle, 8, 0, 256, 0, asm_rows=3)
