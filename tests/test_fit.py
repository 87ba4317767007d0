"""The library's LRS fit (lbm_lrs_fit, host code) against the oracle's
plain normal-equation fit (Sec. 4.4), and its error handling."""
import numpy as np
import pytest

import oracle
from test_oracle_history import _stable_model, _trajectory


@pytest.fixture(scope="module")
def lbm():
    from paper_2609_32892_amd import lbm as m
    m.lib()
    return m


@pytest.mark.parametrize("h,nq,lam,given", [(0, 2, 0.0, True), (2, 3, 0.7, False), (5, 12, 3.0, False),
                                             (1, 1, 0.1, True)])
def test_fit_matches_oracle(lbm, h, nq, lam, given):
    rng = np.random.default_rng(10 + h + nq)
    s = 0.5 + rng.random(nq)
    C_true = _stable_model(h, nq, rng)
    q, qs = _trajectory(h, nq, 400, C_true, s, 0.05, rng)
    Co, muo, So, so = oracle.lrs_fit(q, qs, h, lam, scale=s if given else None)
    C, mu, S, s2 = lbm.lrs_fit(qs, q - qs, h, lam, scale=s if given else None)
    assert np.allclose(s2, so, rtol=1e-13)
    assert np.allclose(C, Co, rtol=0, atol=1e-9 * np.max(np.abs(Co)))
    assert np.allclose(mu, muo, rtol=0, atol=1e-10)
    assert np.allclose(S, So, rtol=1e-8, atol=1e-14)


def test_fit_skipped_steps_use_predictor(lbm):
    """A step flagged as skipped (bit 1) enters the history with q = q*."""
    rng = np.random.default_rng(3)
    h, nq = 2, 2
    s = np.ones(nq)
    q, qs = _trajectory(h, nq, 200, _stable_model(h, nq, rng), s, 0.05, rng)
    flags = np.zeros(len(q), dtype=np.int32)
    flags[[20, 77, 150]] = 2
    qc = q.copy()
    qc[flags == 2] = qs[flags == 2]
    Co, muo, So, _ = oracle.lrs_fit(qc, qs, h, 0.5, scale=s)
    C, mu, S, _ = lbm.lrs_fit(qs, q - qs, h, 0.5, scale=s, flags=flags)
    assert np.allclose(C, Co, rtol=0, atol=1e-9 * np.max(np.abs(Co)))
    assert np.allclose(S, So, rtol=1e-8)


def test_fit_errors(lbm):
    q = np.ones((10, 2))
    with pytest.raises(lbm.LbmError):          # too few steps for h
        lbm.lrs_fit(q, 0 * q, 9, 1.0)
    with pytest.raises(lbm.LbmError):          # singular normal matrix without a penalty
        lbm.lrs_fit(q, 0 * q, 1, 0.0)
    with pytest.raises(lbm.LbmError):          # negative penalty
        lbm.lrs_fit(q, 0 * q, 1, -1.0)
    C, mu, S, s = lbm.lrs_fit(q, 0 * q, 1, 1.0)   # constant data: fine with a penalty
    assert np.all(np.isfinite(C)) and np.allclose(s, 1.0)
