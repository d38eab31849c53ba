"""Pins of the oracle's Wilson-Dirac operator (Schwinger Model subsection of the paper)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import dirac
from oracle.dirac import dirac_matrix, sigma3_full


def free_field_eigs(nt, nx, m0, phi=(0.0, 0.0)):
    """Closed form for constant links U_mu = exp(i phi_mu): plane waves with momenta
    p_t = (2k+1) pi / N_t (antiperiodic), p_x = 2 pi k / N_x, shifted by phi_mu, give
    lambda = m0 + sum_mu (1 - cos p_mu) +- i sqrt(sum_mu sin^2 p_mu)."""
    out = []
    for kt in range(nt):
        for kx in range(nx):
            pt = (2 * kt + 1) * np.pi / nt + phi[0]
            px = 2 * np.pi * kx / nx + phi[1]
            re = m0 + (1 - np.cos(pt)) + (1 - np.cos(px))
            im = np.sqrt(np.sin(pt) ** 2 + np.sin(px) ** 2)
            out += [re + 1j * im, re - 1j * im]
    return np.array(out)


def match_spectra(a, b):
    """Max distance after greedy matching (both are multisets of the same size)."""
    b = list(b)
    worst = 0.0
    for z in a:
        d = np.abs(np.array(b) - z)
        i = int(np.argmin(d))
        worst = max(worst, d[i])
        b.pop(i)
    return worst


@pytest.mark.parametrize("nt,nx", [(4, 4), (6, 4), (4, 8)])
def test_free_field_spectrum(nt, nx):
    U = np.ones((2, nt, nx), dtype=complex)
    ev = np.linalg.eigvals(dirac_matrix(U, 0.3).toarray())
    assert match_spectra(ev, free_field_eigs(nt, nx, 0.3)) < 1e-10


@pytest.mark.parametrize("nt,nx", [(4, 6), (8, 4)])
def test_constant_phase_spectrum_fixes_direction_and_dagger(nt, nx):
    phi = (0.37, -0.81)
    U = np.stack([np.full((nt, nx), np.exp(1j * phi[0])), np.full((nt, nx), np.exp(1j * phi[1]))])
    ev = np.linalg.eigvals(dirac_matrix(U, -0.2).toarray())
    assert match_spectra(ev, free_field_eigs(nt, nx, -0.2, phi)) < 1e-10
    # swapping which direction is time changes the spectrum: the pin sees mu-order mistakes
    assert match_spectra(ev, free_field_eigs(nt, nx, -0.2, phi[::-1])) > 1e-3
    # (U on the backward hop instead of U^dagger would break the shifted plane-wave form
    # itself, so the first assertion already pins the conjugation)


def test_sigma3_matches_paper():
    assert np.allclose(dirac.SIGMA3, np.diag([-1.0, 1.0]))
    for s in dirac.SIGMA:
        assert np.allclose(s @ dirac.SIGMA3 + dirac.SIGMA3 @ s, 0)


def test_sigma3_hermiticity_random_links():
    U = np.exp(1j * np.random.default_rng(5).uniform(-np.pi, np.pi, (2, 6, 8)))
    D = dirac_matrix(U, 0.05)
    S = sigma3_full(48)
    diff = (D.conj().T - S @ D @ S)
    assert abs(diff).max() < 1e-15
    ev = np.linalg.eigvals(D.toarray())
    # eigenvalues come in complex-conjugate pairs
    assert match_spectra(ev, np.conj(ev)) < 1e-10


def test_mass_shift_and_gauge_covariance():
    rng = np.random.default_rng(7)
    nt, nx = 6, 4
    U = np.exp(1j * rng.uniform(-np.pi, np.pi, (2, nt, nx)))
    D0 = dirac_matrix(U, 0.0)
    D1 = dirac_matrix(U, 0.7)
    assert abs(D1 - D0 - 0.7 * sp.identity(2 * nt * nx)).max() < 1e-15
    om = np.exp(1j * rng.uniform(-np.pi, np.pi, (nt, nx)))
    Ug = np.stack([om * U[0] * np.conj(np.roll(om, -1, axis=0)),
                   om * U[1] * np.conj(np.roll(om, -1, axis=1))])
    Om = sp.diags(np.repeat(om.ravel(), 2))
    diff = dirac_matrix(Ug, 0.7) - Om @ D1 @ Om.conj().T
    assert abs(diff).max() < 1e-14


def test_antiperiodic_time_periodic_space():
    """A single link of value 1 on a 4x4 lattice: hop coefficients carry the BC signs."""
    nt = nx = 4
    U = np.ones((2, nt, nx), dtype=complex)
    D = dirac_matrix(U, 0.0).toarray()
    # site (t=3, x=1) -> forward t-neighbour is (0, 1) with sign -1: block -1/2 (1 - sigma0) * (-1)
    n, m = 3 * nx + 1, 0 * nx + 1
    assert np.allclose(D[2 * n:2 * n + 2, 2 * m:2 * m + 2], 0.5 * (np.eye(2) - dirac.SIGMA0))
    # site (1, 3) -> forward x-neighbour (1, 0), no sign
    n, m = 1 * nx + 3, 1 * nx + 0
    assert np.allclose(D[2 * n:2 * n + 2, 2 * m:2 * m + 2], -0.5 * (np.eye(2) - dirac.SIGMA1))


def test_plaquette_and_topology_of_generator():
    """Quenched 2D U(1): <cos theta_P> = I1(beta)/I0(beta) up to O(1/V) torus effects;
    the topological charge (1/2pi) sum_P arg U_P is an integer."""
    from scipy.special import iv
    for beta, L in ((2.0, 32), (6.0, 32)):
        th = synth.gen_theta(L, L, beta, 300, 11)
        tp = synth.plaquette_angles(th)
        plaq = np.mean(np.cos(tp))
        expect = iv(1, beta) / iv(0, beta)
        var = (1 + iv(2, beta) / iv(0, beta)) / 2 - expect ** 2
        assert abs(plaq - expect) < 6 * np.sqrt(var / (L * L)) + 0.01
        q = np.sum(np.angle(np.exp(1j * tp))) / (2 * np.pi)
        assert abs(q - round(q)) < 1e-9


def test_dirac_at_sites_plane_wave_closed_form():
    """Constant links U_mu = exp(i phi_mu), psi = exp(i (p_t t + p_x x)) chi with an antiperiodic
    momentum p_t: D psi = M psi with M = m0 + sum_mu (1 - cos q_mu) + i sum_mu sigma_mu sin q_mu,
    q_mu = p_mu + phi_mu, at every site including both boundaries."""
    nt, nx, m0, phi = 8, 12, 0.21, (0.3, -0.7)
    U = np.empty((2, nt, nx), dtype=complex)
    U[0], U[1] = np.exp(1j * phi[0]), np.exp(1j * phi[1])
    pt, px = 3 * np.pi / nt, 2 * np.pi * 5 / nx
    chi = np.array([0.4 - 0.2j, -1.1 + 0.7j])
    T, X = np.meshgrid(np.arange(nt), np.arange(nx), indexing="ij")
    psi = np.exp(1j * (pt * T + px * X))[..., None] * chi
    qt, qx = pt + phi[0], px + phi[1]
    M = ((m0 + 2 - np.cos(qt) - np.cos(qx)) * np.eye(2)
         + 1j * (np.sin(qt) * dirac.SIGMA0 + np.sin(qx) * dirac.SIGMA1))
    got = dirac.dirac_at_sites(U, m0, psi, T.ravel(), X.ravel())
    want = psi[T.ravel(), X.ravel()] @ M.T
    assert np.abs(got - want).max() < 1e-13


def test_dirac_at_sites_agrees_with_matrix_on_random_links():
    nt, nx = 6, 10
    rng = np.random.default_rng(17)
    U = np.exp(1j * rng.uniform(-np.pi, np.pi, (2, nt, nx)))
    psi = rng.standard_normal((nt, nx, 2)) + 1j * rng.standard_normal((nt, nx, 2))
    D = dirac_matrix(U, -0.3)
    want = (D @ psi.reshape(-1)).reshape(nt, nx, 2)
    T, X = np.meshgrid(np.arange(nt), np.arange(nx), indexing="ij")
    got = dirac.dirac_at_sites(U, -0.3, psi, T.ravel(), X.ravel()).reshape(nt, nx, 2)
    assert np.abs(got - want).max() < 1e-13
