"""proxsdp_project_psd_noalloc (the library's static device scratch instead of
a workspace) against proxsdp_project_psd on the same inputs: two calls in a
row, the second smaller, plus the exact small-n path and the refusals."""
import numpy as np
import pytest

import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(torch, n, rpos, seed):
    lam = I.lowrank_plus_negative_spectrum(n, rpos, seed)
    S = I.random_symmetric(n, lam, seed)
    return torch.tensor(S, device="cuda"), float(np.abs(lam).max())


def test_noalloc_matches_workspace_entry_point(torch_cuda):
    from paper_1810_05231_amd import project_psd, project_psd_noalloc
    torch = torch_cuda
    # (n, r, positive eigenvalues, seed): a larger call, then a smaller one on
    # the same scratch, then the one-workgroup exact path (n <= 64, r = 0)
    for n, r, rpos, seed in [(900, 16, 12, 0), (300, 8, 5, 1), (50, 0, 7, 2)]:
        print("noalloc case", n, r, rpos, seed, flush=True)
        St, scale = _case(torch, n, rpos, seed)
        P_ref, ev_ref, vec_ref, rank_ref = project_psd(St, r, tol=1e-12, want_vectors=True)
        P = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
        P2, ev, vec, rank = project_psd_noalloc(St, r, tol=1e-12, P=P, want_vectors=True)
        torch.cuda.synchronize()
        dP = float((P2 - P_ref).abs().max())
        print("  max |P - P_ref|", dP, "scale", scale, flush=True)
        assert dP <= 1e-12 * scale
        assert np.abs(ev - ev_ref).max() <= 1e-12 * scale
        assert rank == rank_ref
        # eigenvectors up to sign
        sgn = np.sign(np.sum(vec * vec_ref, axis=0))
        assert np.abs(vec * sgn - vec_ref).max() <= 1e-9


def test_noalloc_refusals(torch_cuda):
    from paper_1810_05231_amd import ProxSDPError, project_psd_noalloc
    from paper_1810_05231_amd import _lib as L
    torch = torch_cuda
    S = torch.zeros((100, 100), dtype=torch.float64, device="cuda")
    with pytest.raises(ProxSDPError) as e:        # exact projection above n = 64
        project_psd_noalloc(S, 0)
    assert e.value.code == L.PROXSDP_ERR_UNSUPPORTED
    with pytest.raises(ProxSDPError) as e:        # 45 MB of scratch > 32 MiB
        project_psd_noalloc(torch.zeros((5000, 5000), dtype=torch.float64, device="cuda"), 48)
    assert e.value.code == L.PROXSDP_ERR_WORKSPACE
