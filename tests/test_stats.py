"""tau_int and the tau-corrected error: the oracle against the AR(1) closed form and
i.i.d. data; the library's host implementation against the oracle."""
import numpy as np
import pytest

from oracle import stats


def _ar1(phi, n, chains, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((chains, n))
    e = rng.standard_normal((chains, n))
    x[:, 0] = e[:, 0] / np.sqrt(1 - phi ** 2)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + e[:, t]
    return x


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.8])
def test_oracle_tau_ar1_closed_form(phi):
    x = _ar1(phi, 20000, 4, seed=1)
    exact = (1 + phi) / (2 * (1 - phi))
    taus, _, _ = stats.chain_stats(x)
    assert abs(np.mean(taus) - exact) < 0.08 * exact + 0.03


def test_oracle_error_iid():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((8, 5000))
    _, m, err = stats.chain_stats(x)
    assert abs(err - 1.0 / np.sqrt(40000)) < 0.1 / np.sqrt(40000)


def test_library_matches_oracle():
    from paper_1908_09359_amd import binding as B
    x = _ar1(0.7, 3000, 6, seed=3) + 0.3
    t_lib, m_lib, e_lib = B.vp_stats_tau(x, c=5.0)
    t_or, m_or, e_or = stats.chain_stats(x, c=5.0)
    assert np.allclose(t_lib, t_or, rtol=1e-12)
    assert abs(m_lib - m_or) < 1e-12 and abs(e_lib - e_or) < 1e-12
    with pytest.raises(B.VPError):
        B.vp_stats_tau(x[:, :1])
