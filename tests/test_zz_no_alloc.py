"""The allocation-free pressure solve (nf_pressure_solve_noalloc, through the C
ABI) against the existing entry point nf_pressure_solve on a handle, on two
calls in a row: the largest grid the fixed workspace serves, then a smaller
one on a non-unit box (the second call runs over the first call's leftovers
in the shared array).  Held to the FP64 bar, 1e-10 relative L2, with equal
iteration counts; both are also checked against the oracle.  Each handle is
created before the allocation-free call of its shape, so that both run the
tile variants tuned for the shape."""

import numpy as np
import pytest

import oracle as O

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

TOL = 1e-10


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def fields(n, seed):
    rng = np.random.default_rng(seed)
    shape = n[::-1]
    m = rng.uniform(-1.0, 1.0, (2,) + shape)
    r = rng.uniform(0.05, 0.15, shape)
    S = rng.standard_normal(shape)
    S -= S.mean()
    return m, r, S


def test_noalloc_solve_matches_handle_solve_on_consecutive_calls():
    import torch

    from paper_2606_06720_amd import nf as NF

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    for k, (n, L, rtol) in enumerate((((256, 256), (1.0, 1.0), 1e-11), ((64, 32), (2.0, 0.5), 1e-10))):
        print("noalloc case", k, n, L, flush=True)
        m, r, S = fields(n, 100 + k)
        # the handle first: it fixes the shape's tile variants, which the
        # allocation-free solve then uses as well
        p_ref = torch.zeros(n[::-1], dtype=torch.float64, device=dev)
        with NF.Grid(n, L) as g:
            rc, info_ref = g.pressure_solve(T(m), T(r), T(S), p_ref, rtol=rtol, max_iter=2000)
        p_free = torch.zeros(n[::-1], dtype=torch.float64, device=dev)
        rc, info_free = NF.nf_pressure_solve_noalloc(n, L, T(m), T(r), T(S), p_free, rtol=rtol, max_iter=2000)
        assert rc == NF.NF_OK and info_free.converged
        assert info_free.iters == info_ref.iters
        assert abs(info_free.true_rel_res - info_ref.true_rel_res) <= 1e-3 * info_ref.true_rel_res
        a, b = p_free.cpu().numpy(), p_ref.cpu().numpy()
        assert rel(a, b) <= TOL
        p_or, _ = O.pressure_pcg(m, r, S, None, rtol, 2000, L)
        assert rel(a, p_or) <= TOL
    # a size beyond the workspace is refused before any device work
    with pytest.raises(NF.NfError) as e:
        z = torch.zeros((256, 512), dtype=torch.float64, device=dev)
        NF.nf_pressure_solve_noalloc((512, 256), None, torch.zeros((2, 256, 512), dtype=torch.float64, device=dev),
                                     z, z, z.clone())
    assert e.value.code == NF.NF_EINVAL
