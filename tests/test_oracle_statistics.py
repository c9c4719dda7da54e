"""Loose statistical sanity checks of the dynamics (not parity): KPZ power-law
roughening for p > 0 = q (Sec. I-A), with growth exponent beta near 0.24 in
2+1 dimensions."""
import numpy as np
import pytest


@pytest.mark.slow
def test_kpz_growth_exponent(orc):
    L = 512
    st = orc.flat(L, L, track_heights=False)
    ts, w2 = [], []
    t = 0
    for target in [16, 23, 32, 45, 64, 91, 128, 181, 256]:
        orc.run(st, target - t, 0.75, 0.0, seed=20160601)
        t = target
        ts.append(t)
        w2.append(orc.moments(st)[3])
    slope = np.polyfit(np.log(ts), np.log(w2), 1)[0]
    # 2 beta ~ 0.48; generous band for a single small realization
    assert 0.36 <= slope <= 0.60, slope


@pytest.mark.slow
def test_edwards_wilkinson_logarithmic_roughening(orc):
    """p = q falls into the Edwards-Wilkinson class (Sec. I-A): W^2 grows like
    a + b ln t, far below the KPZ power law."""
    L = 512
    st = orc.flat(L, L, track_heights=False)
    ts, w2 = [], []
    t = 0
    for target in [8, 16, 32, 64, 128, 256, 512]:
        orc.run(st, target - t, 0.5, 0.5, seed=11)
        t = target
        ts.append(t)
        w2.append(orc.moments(st)[3])
    lt = np.log(ts)
    b, a = np.polyfit(lt, w2, 1)
    resid = np.asarray(w2) - (a + b * lt)
    assert b > 0.05 and np.max(np.abs(resid)) < 0.05 * np.max(w2), (a, b, resid)
    assert np.polyfit(lt, np.log(w2), 1)[0] < 0.2  # KPZ would give ~0.4-0.5
    incr = np.diff(w2)
    assert 0.4 < incr[-1] / incr[0] < 2.5  # equal steps per doubling of t
