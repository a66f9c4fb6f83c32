"""Pins for the characteristic decomposition of the oracle's TVB limiter
(Section 5.3): the left and right eigenvector matrices are checked against
the flux Jacobian of Eq. 2.2, which the test forms on its own by complex-step
differentiation of the physical flux (no eigen-formula is shared), and the
per-edge limiting step is checked to give back the deviation it was handed
when no characteristic component is cut."""
import numpy as np
import pytest

from oracle.swe import char_left, char_minmod, char_right

G = 9.81


def _states(n, seed):
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.05, 3.0, n)
    u = rng.normal(0.0, 1.5, n)
    v = rng.normal(0.0, 1.5, n)
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    return h, u, v, np.cos(th), np.sin(th)


def _normal_flux(q, ex, ey):
    """F(q) ex + G(q) ey of the conservative shallow water system (Eq. 2.2)."""
    h, hu, hv = q
    un = (hu * ex + hv * ey) / h
    return np.array([h * un, hu * un + 0.5 * G * h * h * ex, hv * un + 0.5 * G * h * h * ey])


def _jacobian(h, u, v, ex, ey):
    """dF_n/dq by complex-step differentiation (exact to rounding)."""
    q = np.array([h, h * u, h * v], dtype=complex)
    J = np.zeros((3, 3))
    step = 1e-30
    for b in range(3):
        qp = q.copy()
        qp[b] += 1j * step
        J[:, b] = _normal_flux(qp, ex, ey).imag / step
    return J


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_left_right_are_inverse(seed):
    h, u, v, ex, ey = _states(200, seed)
    c = np.sqrt(G * h)
    L = char_left(u, v, c, ex, ey)
    R = char_right(u, v, c, ex, ey)
    eye = np.broadcast_to(np.eye(3), L.shape)
    assert np.max(np.abs(R @ L - eye)) < 1e-12
    assert np.max(np.abs(L @ R - eye)) < 1e-12


@pytest.mark.parametrize("seed", [3, 4])
def test_left_right_diagonalise_the_flux_jacobian(seed):
    """L A_n R = diag(un - c, un, un + c): the rows of L and the columns of R
    are the eigenvectors of the Jacobian of F ex + G ey, in that order."""
    h, u, v, ex, ey = _states(50, seed)
    c = np.sqrt(G * h)
    L = char_left(u, v, c, ex, ey)
    R = char_right(u, v, c, ex, ey)
    for k in range(h.size):
        A = _jacobian(h[k], u[k], v[k], ex[k], ey[k])
        D = L[k] @ A @ R[k]
        un = u[k] * ex[k] + v[k] * ey[k]
        want = np.diag([un - c[k], un, un + c[k]])
        scale = abs(un) + c[k]
        assert np.max(np.abs(D - want)) < 1e-12 * scale, (k, D, want)
        # and each column of R is an eigenvector of A itself
        for j, lam in enumerate((un - c[k], un, un + c[k])):
            assert np.max(np.abs(A @ R[k][:, j] - lam * R[k][:, j])) < 1e-12 * scale * (1 + abs(lam))


def test_unlimited_edge_returns_its_deviation():
    """When minmod returns a1 in every component (neighbour increment of the
    same sign and larger), the limited deviation R m~ = R L dev is the
    deviation itself; the TVB bypass (|a1| <= M d^2) does the same."""
    n = 300
    h, u, v, ex, ey = _states(n, 5)
    c = np.sqrt(G * h)
    rng = np.random.default_rng(6)
    dev = rng.normal(0.0, 0.1, (3, n))
    L = char_left(u, v, c, ex, ey)
    R = char_right(u, v, c, ex, ey)
    a1 = np.einsum("nab,bn->an", L, dev)
    # a neighbour increment whose characteristic components are 2x those of
    # dev, so nu * a2 has the same signs and larger magnitudes
    dbar = np.einsum("nab,bn->an", R, 2.0 * a1)
    out, kept = char_minmod(u, v, c, ex, ey, dev, dbar, 1.5, np.zeros(n))
    assert np.all(kept)
    assert np.max(np.abs(out - dev)) < 1e-13
    out2, kept2 = char_minmod(u, v, c, ex, ey, dev, -dbar, 1.5, np.full(n, 1e9))
    assert np.all(kept2)
    assert np.max(np.abs(out2 - dev)) < 1e-13


def test_limited_edge_cuts_each_characteristic_field():
    """A neighbour increment of opposite sign in one characteristic field
    zeroes exactly that field: the output is dev minus a1_j r_j."""
    n = 100
    h, u, v, ex, ey = _states(n, 8)
    c = np.sqrt(G * h)
    rng = np.random.default_rng(9)
    dev = rng.normal(0.0, 0.1, (3, n))
    L = char_left(u, v, c, ex, ey)
    R = char_right(u, v, c, ex, ey)
    a1 = np.einsum("nab,bn->an", L, dev)
    for j in range(3):
        a2 = 2.0 * a1
        a2[j] = -a1[j]
        dbar = np.einsum("nab,bn->an", R, a2)
        out, kept = char_minmod(u, v, c, ex, ey, dev, dbar, 1.5, np.zeros(n))
        assert not np.any(kept)
        want = dev - R[:, :, j].T * a1[j][None, :]
        assert np.max(np.abs(out - want)) < 1e-13
