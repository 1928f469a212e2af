"""The allocation-free projected SVD (mqh_proj_svd_noalloc) against mqh_proj_svd.

Both run the same kernel on the same device inputs, so the outputs agree bit
for bit; two calls in a row (the second smaller) check that the shared
workspace keeps no state that the next call depends on.  The leading Ritz
values are also compared with the oracle's projected SVD (1e-12 relative).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _bidiag(ell, seed):
    # Krylov-like scalars: a decaying bidiagonal with a few close values
    rng = np.random.default_rng(seed)
    alpha = np.exp(-np.linspace(0.0, 12.0, ell)) * (1.0 + 0.1 * rng.random(ell))
    beta = np.exp(-np.linspace(0.0, 12.0, ell + 1)) * (0.5 + 0.1 * rng.random(ell + 1))
    beta[0] = 3.0
    return alpha, beta


def test_noalloc_matches_allocating_call(orc):
    import torch

    from paper_2511_09798_amd import mqhelm as mq

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for ell, seed in ((300, 1), (120, 2)):
        a, b = _bidiag(ell, seed)
        da = torch.from_numpy(a).to(dev)
        db = torch.from_numpy(b).to(dev)
        say("reference mqh_proj_svd, ell", ell)
        sv0, ft0, V0 = mq.mqh_proj_svd(da, db, want_v=True, stream=stream)
        say("mqh_proj_svd_noalloc with V, ell", ell)
        sv1 = torch.empty(ell, dtype=torch.float64, device=dev)
        ft1 = torch.empty(ell + 1, dtype=torch.float64, device=dev)
        V1 = torch.empty((ell, ell), dtype=torch.float64, device=dev)
        mq.mqh_proj_svd_noalloc(da, db, sv1, ft1, V1, stream=stream)
        say("mqh_proj_svd_noalloc without V, ell", ell)
        sv2 = torch.empty(ell, dtype=torch.float64, device=dev)
        ft2 = torch.empty(ell + 1, dtype=torch.float64, device=dev)
        mq.mqh_proj_svd_noalloc(da, db, sv2, ft2, None, stream=stream)
        torch.cuda.synchronize()
        r0 = [t.cpu().numpy() for t in (sv0, ft0, V0)]
        assert np.array_equal(sv1.cpu().numpy(), r0[0])
        assert np.array_equal(ft1.cpu().numpy(), r0[1])
        assert np.array_equal(V1.cpu().numpy(), r0[2])
        assert np.array_equal(sv2.cpu().numpy(), r0[0])
        assert np.array_equal(ft2.cpu().numpy(), r0[1])
        s_o, f_o, _ = orc.proj_svd(a, b)
        assert np.max(np.abs(r0[0][:10] - s_o[:10]) / s_o[:10]) < 1e-12
        assert np.max(np.abs(np.abs(r0[1][:10]) - np.abs(f_o[:10]))) <= 1e-12 * b[0]


def test_noalloc_rejects_oversize():
    import torch

    from paper_2511_09798_amd import mqhelm as mq

    dev = torch.device("cuda:0")
    ell = mq.MQH_NOALLOC_MAX_ELL + 1
    a = torch.ones(ell, dtype=torch.float64, device=dev)
    b = torch.ones(ell + 1, dtype=torch.float64, device=dev)
    with pytest.raises(mq.MQHError) as err:
        mq.mqh_proj_svd_noalloc(a, b, torch.empty_like(a), torch.empty_like(b))
    assert err.value.code == mq.MQH_EINVAL
