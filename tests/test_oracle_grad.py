"""Pins of the reference gradients (forward-mode dual numbers through the
FP64 rollout) against central finite differences and a closed form.

The differentiable workload: closed loop, per-agent gains, loss =
sum ||p_T - target||^2 + 1e-4 * J_T.  Finite differences run in the
target-centred frame, which the dynamics allow exactly (nothing but the
controller's waypoint error sees absolute position), and which removes the
cancellation of large coordinates from the difference quotient.
"""
import numpy as np
import pytest

from paper_2308_12698_amd import inputs as I

H = 1e-6


def loss_and_seed(final, target, w):
    d = final[0:3] - target
    L = np.sum(d * d, axis=0) + w * final[29]
    gN = np.zeros_like(final)
    gN[0:3] = 2.0 * d
    gN[29] = w
    return L, gN


def centred(sw):
    tgt = sw.extra["target"].astype(np.float64)
    s = sw.state.astype(np.float64).copy()
    s[0:3] -= tgt
    wp = sw.wp.astype(np.float64) - tgt[None]
    return s, wp, np.zeros_like(tgt)


@pytest.fixture(scope="module")
def diff_case():
    sw = I.subset(I.config4(n=4096), np.array([3, 1000, 2047, 4000]))
    return sw


def test_dual_gradient_matches_central_differences(oracle, diff_case):
    sw = diff_case
    s0, wp, tgt = centred(sw)
    gains = sw.gains.astype(np.float64)
    n, T, dt, w = sw.n, sw.n_steps, sw.dt, sw.extra["cost_weight"]
    kw = dict(wp=wp, gains=gains, threads=1)
    fin, jac = oracle.jacobian(s0, sw.types, sw.glob, dt, T, **{k: v for k, v in kw.items() if k != "threads"})
    _, gN = loss_and_seed(fin, tgt, w)
    g_dual = np.einsum("ar,arc->ac", gN[:30].T, jac)             # [n, 39]

    def L_of(s, g):
        f = oracle.rollout(s, sw.types, sw.glob, 1, dt, T, wp=wp, gains=g, threads=1)
        return loss_and_seed(f, tgt, w)[0]

    g_fd = np.zeros((n, 39))
    for c in range(39):
        sp, sm = s0.copy(), s0.copy()
        gp, gm = gains.copy(), gains.copy()
        if c < 30:
            sp[c] += H; sm[c] -= H
        else:
            gp[c - 30] += H; gm[c - 30] -= H
        g_fd[:, c] = (L_of(sp, gp) - L_of(sm, gm)) / (2 * H)
    for a in range(n):
        for blk in (slice(0, 30), slice(30, 39)):
            num = np.linalg.norm(g_dual[a, blk] - g_fd[a, blk])
            assert num <= 1e-5 * np.linalg.norm(g_dual[a, blk]), (a, blk, g_dual[a, blk], g_fd[a, blk])


def test_dual_jacobian_columns_match_differences(oracle, diff_case):
    """Every column of d x_N / d (x0, gains), short rollout, two agents."""
    sw = I.subset(diff_case, np.array([0, 2]))
    s0, wp, _ = centred(sw)
    gains = sw.gains.astype(np.float64)
    T, dt = 60, sw.dt
    fin, jac = oracle.jacobian(s0, sw.types, sw.glob, dt, T, wp=wp, gains=gains)
    ref = oracle.rollout(s0, sw.types, sw.glob, 1, dt, T, wp=wp, gains=gains, threads=1)
    assert np.array_equal(fin, ref)
    for c in range(39):
        sp, sm = s0.copy(), s0.copy()
        gp, gm = gains.copy(), gains.copy()
        if c < 30:
            sp[c] += H; sm[c] -= H
        else:
            gp[c - 30] += H; gm[c - 30] -= H
        fp = oracle.rollout(sp, sw.types, sw.glob, 1, dt, T, wp=wp, gains=gp, threads=1)
        fm = oracle.rollout(sm, sw.types, sw.glob, 1, dt, T, wp=wp, gains=gm, threads=1)
        col = ((fp - fm) / (2 * H))[:30]                          # [30, n]
        for a in range(2):
            # truncation ~ h^2 f''' plus cancellation eps |x_N| / h per row
            tol = 1e-5 * max(np.abs(jac[a, :, c]).max(), 1e-3) + 50 * 2.2e-16 * np.abs(ref[:30, a]) / H
            assert np.all(np.abs(jac[a, :, c] - col[:, a]) <= tol), (c, a)


def test_linear_special_case_gradient(oracle):
    """Motors held off (speed limit 0), no drag: p_T = p_0 + v_0 T - g T^2/2,
    so dp_T/dp_0 = I, dp_T/dv_0 = T I and the gains have no influence."""
    t = I.base_type(w_max=0.0, drag=0.0)
    t["w_ref"] = np.float32(0.0)
    s0 = I.hover_state(np.array([[1.0], [2.0], [30.0]])).astype(np.float64)
    s0[3:6, 0] = (0.3, -0.2, 0.1)
    T, dt = 200, 2e-3
    wp = np.array([[[1.5], [2.5], [31.0]]])
    fin, jac = oracle.jacobian(s0, [t], I.globals_f32(), dt, T, wp=wp)
    j = jac[0]
    assert np.allclose(j[0:3, 0:3], np.eye(3), atol=1e-12)
    assert np.allclose(j[0:3, 3:6], T * dt * np.eye(3), atol=1e-12)
    assert np.abs(j[0:3, 6:]).max() <= 1e-12
    g32 = float(np.float32(9.81))
    assert fin[2, 0] == pytest.approx(30.0 + 0.1 * 0.4 - 0.5 * g32 * 0.4 ** 2, abs=1e-12)
