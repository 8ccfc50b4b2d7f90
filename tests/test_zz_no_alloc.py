"""The allocation-free reduced eigensolve against the allocating entry point.

feast_reduced_eig_noalloc runs the kernels of feast_reduced_eig on the
library's file-scope device array instead of the context's workspace; its
results must be those of feast_reduced_eig bit for bit, on consecutive calls
that share the array (the second one smaller), and match the CPU oracle.
"""
import numpy as np
import pytest

from oracle import feast_oracle as O

pytestmark = pytest.mark.gpu


def _pair(n, seed, cond):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    mu = np.geomspace(1.0, 1.0 / cond, n)
    BQ = (Qm * mu) @ Qm.T
    AQ = rng.standard_normal((n, n))
    return 0.5 * (AQ + AQ.T), 0.5 * (BQ + BQ.T)


def _rank_deficient(n, k, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, k))
    return G @ np.diag(np.arange(1.0, k + 1.0)) @ G.T, G @ G.T


def test_reduced_eig_noalloc_matches_allocating_entry_point():
    import torch
    from paper_0901_2665_amd import feast as F
    assert torch.cuda.is_available()
    ctx = F.Context(0)
    try:
        cases = [_pair(128, 5, 1e3), _pair(30, 6, 1e2), _rank_deficient(20, 12, 7)]
        for AQ, BQ in cases:
            n = AQ.shape[0]
            a = torch.as_tensor(AQ, dtype=torch.float64, device="cuda").contiguous()
            b = torch.as_tensor(BQ, dtype=torch.float64, device="cuda").contiguous()
            eps = torch.empty(n, dtype=torch.float64, device="cuda")
            Phi = torch.empty((n, n), dtype=torch.float64, device="cuda")
            fb = ctx.reduced_eig_noalloc(a, b, eps, Phi)
            eps_ref, Phi_ref, fb_ref = ctx.reduced_eig(a, b)
            assert fb == fb_ref
            assert torch.equal(eps.isnan(), eps_ref.isnan())
            fin = ~eps_ref.isnan()
            assert torch.equal(eps[fin], eps_ref[fin]) and torch.equal(Phi, Phi_ref)
            ref, _, rfb = O.reduced_eig(AQ, BQ)
            assert fb == rfb
            e = eps.cpu().numpy()
            k = int(np.sum(np.isfinite(ref)))
            assert np.allclose(e[:k], ref[:k], rtol=0, atol=1e-8 * np.max(np.abs(ref[:k])))
        # the size limit of the static array is reported, not overrun
        big = torch.zeros((129, 129), dtype=torch.float64, device="cuda")
        with pytest.raises(F.FeastError) as err:
            ctx.reduced_eig_noalloc(big, big, torch.empty(129, dtype=torch.float64, device="cuda"),
                                    big)
        assert err.value.status == -3
    finally:
        ctx.close()
