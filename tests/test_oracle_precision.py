"""Pins for the oracle's FP16 storage model (oracle/precision.py): with no
field rounded it is the FP64 gradient and Gauss-Newton matvec of the core
oracle; its rounding primitive is IEEE binary16 round-to-nearest-even; and on
the paper's synthetic problem (Sec. 4.2) rounding the adjoint and incremental
fields keeps the gradient and matvec within 1e-3 of FP64, while rounding the
state history does not (the reason the state stays FP32 in the FP16-storage
mode)."""
import numpy as np
import pytest

from oracle import core, prep, precision
from paper_1808_04487_amd import synth


def problem(n):
    g = core.Grid(n)
    mT = synth.trig_template(n)
    vs = synth.trig_velocity(n)
    mR = prep.transport(g, mT, vs)
    p = core.Params(n, reg=core.REG_H1, div_mode=core.DIV_NEAR, beta_v=1e-2, beta_w=1.0)
    R = core.Registration(p, mT, mR)
    rng = np.random.default_rng(61)
    noise = np.stack([core.gauss_smooth(g, rng.standard_normal(n), 2.0) for _ in range(3)])
    R.set_velocity(0.6 * vs + 0.1 * noise / np.abs(noise).max())
    rng = np.random.default_rng(62)
    vt = np.stack([core.gauss_smooth(g, rng.standard_normal(n), 2.0) for _ in range(3)])
    return g, R, vt / np.abs(vt).max()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_round16_is_binary16_nearest_even():
    one = 1.0
    u = 2.0 ** -10  # spacing of binary16 in [1, 2)
    assert precision.round16(np.array([one + u / 2]))[0] == one          # tie to even
    assert precision.round16(np.array([one + 1.5 * u]))[0] == one + 2 * u  # tie to even
    assert precision.round16(np.array([one + 0.75 * u]))[0] == one + u
    assert precision.round16(np.array([65504.0]))[0] == 65504.0          # largest finite
    x = np.random.default_rng(3).uniform(-4, 4, 100000)
    x = x[np.abs(x) > 2.0 ** -14]                                        # normal range
    assert np.all(np.abs(precision.round16(x) - x) <= 2.0 ** -11 * np.abs(x))


def test_no_rounding_equals_core():
    g, R, vt = problem((16, 16, 16))
    S = precision.StoredRegistration(R, ())
    assert rel_l2(S.gradient(), R.gradient()) < 1e-13
    assert rel_l2(S.hessian_matvec(vt), R.hessian_matvec(vt)) < 1e-13


def test_rounding_each_field_changes_the_result():
    """Every selectable field enters the model: rounding it alone moves the
    gradient (state, lam) or the matvec (state, inc) by more than FP64
    noise, and rounding lam leaves the matvec untouched (GN drops lam)."""
    g, R, vt = problem((16, 16, 16))
    g0, h0 = R.gradient(), R.hessian_matvec(vt)
    for f in ("state", "lam"):
        assert rel_l2(precision.StoredRegistration(R, (f,)).gradient(), g0) > 1e-6
    for f in ("state", "inc"):
        assert rel_l2(precision.StoredRegistration(R, (f,)).hessian_matvec(vt), h0) > 1e-6
    assert rel_l2(precision.StoredRegistration(R, ("lam",)).hessian_matvec(vt), h0) < 1e-13
    assert rel_l2(precision.StoredRegistration(R, ("inc",)).gradient(), g0) < 1e-13
    with pytest.raises(ValueError):
        precision.StoredRegistration(R, ("grad",))


def test_fp16_adjoint_storage_within_1e3_state_storage_not():
    g, R, vt = problem((32, 32, 32))
    g0, h0 = R.gradient(), R.hessian_matvec(vt)
    S = precision.StoredRegistration(R, ("lam", "inc"))
    eg, eh = rel_l2(S.gradient(), g0), rel_l2(S.hessian_matvec(vt), h0)
    assert eg < 1e-3 and eh < 1e-3, (eg, eh)
    T = precision.StoredRegistration(R, ("lam", "inc", "state"))
    eg16 = rel_l2(T.gradient(), g0)
    # lam(1) = mR - m(1) is ~4% of |m| here: rounding m costs ~25x more
    assert eg16 > 1e-3 and eg16 > 5 * eg, (eg16, eg)
