"""The allocation-free matrix-powers entry point (ssp_mpk_noalloc) against
ssp_mpk, through the C ABI: two calls in a row on one handle, the second on
a smaller problem, each equal to ssp_mpk's basis and moments bit for bit
(the same kernels; only the control block and the partial sums live in the
library's static scratch), and the basis equal to the oracle's as well."""
import numpy as np
import pytest

import oracle
from paper_2501_03743_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(H, kind, shape, s, seed, csr_form):
    csr = wl.stencil_csr(kind, shape)
    n = csr[0].shape[0] - 1
    r = np.random.default_rng(seed).standard_normal(n)
    if csr_form:
        A = H.matrix_csr(*[torch.from_numpy(a).cuda() for a in csr])
    else:
        A = H.matrix_stencil(kind, shape)
    rd = torch.from_numpy(r).cuda()
    P_ref, vm_ref = H.mpk(A, rd, s)
    P = torch.full((2 * s, n), np.nan, dtype=torch.float64, device="cuda")
    P_na, vm_na = H.mpk(A, rd, s, P=P, noalloc=True)
    torch.cuda.synchronize()
    # the oracle's operator in the same form (the matrix-free stencil sums a
    # row's terms in the stencil's order, the CSR form in column order)
    op = oracle.Operator("csr", csr=csr) if csr_form else oracle.Operator(kind, shape)
    Pref_o, vmref_o = oracle.mpk_cvm(op, r, s)
    out = (P_na.cpu().numpy(), vm_na, P_ref.cpu().numpy(), vm_ref, Pref_o, vmref_o)
    A.close()
    return out


@pytest.mark.parametrize("csr_form", [True, False])
def test_noalloc_mpk_equals_mpk_twice_second_smaller(csr_form):
    from paper_2501_03743_amd import sstep
    cases = [("3d7", (23, 19, 17), 4, 1), ("2d5", (30, 29), 3, 2)]
    with sstep.Handle(0) as H:
        for kind, shape, s, seed in cases:
            print("[noalloc] %s %s s=%d csr=%s" % (kind, shape, s, csr_form), flush=True)
            P, vm, Pr, vmr, Po, vmo = _case(H, kind, shape, s, seed, csr_form)
            assert np.array_equal(P, Pr), (kind, shape)
            assert np.array_equal(vm, vmr), (kind, shape, vm, vmr)
            assert np.array_equal(P, Po), (kind, shape)
            np.testing.assert_allclose(vm, vmo, rtol=1e-12, atol=0)


def test_noalloc_rejects_invalid_arguments():
    from paper_2501_03743_amd import sstep
    with sstep.Handle(0) as H:
        A = H.matrix_stencil("3d7", (8, 8, 8))
        r = torch.zeros(512, dtype=torch.float64, device="cuda")
        P = torch.empty((2 * 17, 512), dtype=torch.float64, device="cuda")
        with pytest.raises(sstep.SspError):
            H.mpk(A, r, 17, P=P, noalloc=True)
        with pytest.raises(ValueError):
            H.mpk(A, r, 2, noalloc=True)
        A.close()
