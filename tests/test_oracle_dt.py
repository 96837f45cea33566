"""The discrete-time Jacobians of one semi-implicit Euler step, written out from dFD, against
central differences of the step itself computed with the FP64 oracle's forward dynamics.

step(q, qd, tau) = (q + dt qd', qd'), qd' = qd + dt FD(q, qd, tau);
A = d step / d(q, qd) = [[1 + dt^2 Dq, dt 1 + dt^2 Dqd], [dt Dq, 1 + dt Dqd]],
B = d step / dtau = [[dt^2 M^-1], [dt M^-1]], Dq, Dqd, M^-1 from the oracle's analytic dFD.
"""
import numpy as np
import pytest

from paper_2109_06976_amd import synth


def euler_jacobians(Dq, Dqd, Minv, dt):
    n = Dq.shape[0]
    I = np.eye(n)
    A = np.block([[I + dt * dt * Dq, dt * I + dt * dt * Dqd], [dt * Dq, I + dt * Dqd]])
    B = np.vstack([dt * dt * Minv, dt * Minv])
    return A, B


def step(orc, model, q, qd, tau, dt):
    qd1 = qd + dt * orc.fd(model, q, qd, tau)
    return np.concatenate([q + dt * qd1, qd1])


@pytest.mark.parametrize("name", ["chain7", "quad12", "tree5-axes"])
@pytest.mark.parametrize("dt", [0.01, 0.1])
def test_euler_jacobians_match_central_differences(orc, name, dt):
    model = (synth.random_model(np.array([-1, 0, 0, 1, -1], np.int32), 6, "tree5-axes",
                                axes="random") if name == "tree5-axes"
             else synth.model_by_name(name))
    n = model.n
    kn = synth.random_knots(n, 1, 33)
    q, qd, tau = (a[0].astype(float) for a in (kn.q, kn.qd, kn.tau))
    _, Minv, Dq, Dqd = orc.fd_grad(model, q, qd, tau)
    A, B = euler_jacobians(Dq, Dqd, Minv, dt)
    h = 1e-6
    x = np.concatenate([q, qd])
    Afd = np.zeros((2 * n, 2 * n))
    for j in range(2 * n):
        e = np.zeros(2 * n)
        e[j] = h
        xp, xm = x + e, x - e
        Afd[:, j] = (step(orc, model, xp[:n], xp[n:], tau, dt)
                     - step(orc, model, xm[:n], xm[n:], tau, dt)) / (2 * h)
    Bfd = np.zeros((2 * n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        Bfd[:, j] = (step(orc, model, q, qd, tau + e, dt) - step(orc, model, q, qd, tau - e, dt)) \
            / (2 * h)
    np.testing.assert_allclose(A, Afd, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(B, Bfd, rtol=1e-6, atol=1e-9)
