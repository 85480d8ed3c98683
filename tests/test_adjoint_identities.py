"""CPU check of the identities behind the backward sweep of the yield gradient.

The GPU adjoint carries W_s = Im <chi'_s|tau|psi_s> (one real 3-vector per block) instead of the
two spinors.  This test builds both forms in complex128 for random steps and checks that
  * the per-step terms Re <chi'_{n+1}| dU_n/dq_j |psi_n> equal
    q_j (S^2 + C D)(q.W) + C S W_j - S^2 (q x W)_j with W = W_{n+1},
  * W_n = (C^2 - S^2 x) W + 2 S^2 (q.W) q - 2 C S (q x W), here in the tangent-form coefficients
    C^2 (1 - T^2 x), 2 C^2 T^2, C^2 (T^2 - R), C^2 T with T = tan|q|/|q|, R = (T - 1)/x,
  * the initial-state term Re(<chi'_0|+><+|tau_k|->)/w equals (n x W_0)_k / w,
and that the spinor terms are the derivative of f = |<+|psi_N>|^2 (central differences).
Plain linear algebra only: neither the oracle nor the HIP path is involved.
"""
import numpy as np
import pytest

TX = np.array([[0, 1], [1, 0]], complex)
TY = np.array([[0, -1j], [1j, 0]])
TZ = np.array([[1, 0], [0, -1]], complex)
TAU = (TX, TY, TZ)


def step(q):
    x = q @ q
    th = np.sqrt(x)
    C, S = np.cos(th), np.sin(th) / th
    Q = q[0] * TX + q[1] * TY + q[2] * TZ
    return C * np.eye(2) - 1j * S * Q, C, S, (C - S) / x, Q


def eig(P):
    w, v = np.linalg.eigh(P[0] * TX + P[1] * TY + P[2] * TZ)
    return v[:, 1], v[:, 0], w[1]


def f_of(qs, dn_in, up_out):
    psi = dn_in
    for q in qs:
        psi = step(q)[0] @ psi
    return abs(np.vdot(up_out, psi)) ** 2


@pytest.mark.parametrize("s", [1, -1])
def test_three_vector_backward_sweep(s):
    rng = np.random.default_rng(7 + s)
    N, dt = 48, 0.35
    p = np.array([0.3, -0.7, 0.5])
    e = np.sqrt(1 + p[2] ** 2)
    A = rng.normal(size=(N, 2)) * 0.6
    Ain, Aout = rng.normal(size=2) * 0.3, rng.normal(size=2) * 0.3
    qs = [np.array([(p[0] - A[n, 0]) * dt, s * (p[1] - A[n, 1]) * dt, e * dt]) for n in range(N)]
    Pin = np.array([p[0] - Ain[0], s * (p[1] - Ain[1]), e])
    up_in, dn_in, w_in = eig(Pin)
    up_out, _, _ = eig(np.array([p[0] - Aout[0], s * (p[1] - Aout[1]), e]))

    psi = [dn_in]
    for q in qs:
        psi.append(step(q)[0] @ psi[-1])
    alpha = np.vdot(up_out, psi[-1])
    chi = [None] * (N + 1)
    chi[N] = alpha * up_out
    for n in range(N - 1, -1, -1):
        chi[n] = step(qs[n])[0].conj().T @ chi[n + 1]

    ref = np.zeros((N, 2))
    for n, q in enumerate(qs):
        _, C, S, D, Q = step(q)
        for j in range(2):
            dU = q[j] * (-S * np.eye(2) - 1j * D * Q) - 1j * S * TAU[j]
            ref[n, j] = np.real(np.vdot(chi[n + 1], dU @ psi[n]))

    # the spinor terms are the derivative of f (factor 2 of 2 Re)
    f0 = f_of(qs, dn_in, up_out)
    for n in (0, N // 2, N - 1):
        for j in range(2):
            h = 1e-5
            qp = [q.copy() for q in qs]
            qm = [q.copy() for q in qs]
            qp[n][j] += h
            qm[n][j] -= h
            fd = (f_of(qp, dn_in, up_out) - f_of(qm, dn_in, up_out)) / (2 * h)
            assert abs(fd - 2 * ref[n, j]) <= 1e-8 * max(1.0, abs(fd)) + 1e-9 * f0

    W = np.array([np.imag(np.conj(alpha) * np.vdot(up_out, t @ psi[N])) for t in TAU])
    new = np.zeros((N, 2))
    for n in range(N - 1, -1, -1):
        q = qs[n]
        x = q @ q
        th = np.sqrt(x)
        T = np.tan(th) / th
        R = (T - 1) / x
        c2 = np.cos(th) ** 2
        pw, cr = q @ W, np.cross(q, W)
        for j in range(2):
            new[n, j] = c2 * (q[j] * (T * T - R) * pw + T * W[j] - T * T * cr[j])
        W = c2 * (1 - T * T * x) * W + 2 * c2 * T * T * pw * q - 2 * c2 * T * cr
        # the exact-form coefficients give the same rotation
        _, C, S, D, _ = step(q)
        assert np.allclose(c2 * (T * T - R), S * S + C * D, rtol=1e-12, atol=1e-15)
    assert np.max(np.abs(new - ref)) <= 1e-14

    c = np.vdot(chi[0], up_in)
    ref_e = np.array([np.real(c * np.vdot(up_in, TX @ dn_in)), np.real(c * np.vdot(up_in, TY @ dn_in))]) / w_in
    nw = np.cross(Pin / w_in, W) / w_in
    assert np.max(np.abs(nw[:2] - ref_e)) <= 1e-14
