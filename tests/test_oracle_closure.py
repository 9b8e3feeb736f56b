"""Pins of the oracle's SPH kernels and thermodynamic closure against
closed forms, quadrature and finite differences (Sec. 2.1 of the paper)."""
import numpy as np
import pytest
from scipy import integrate

import oracle as O

KERNELS = [O.KERNEL_LUCY, O.KERNEL_CUBIC]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("h", [1.0, 2.5, 3.7])
def test_kernel_normalised(kernel, h):
    # int W d^3r = 1 (Sec. 2.1.1: the kernel is normalised)
    val, err = integrate.quad(lambda r: 4 * np.pi * r * r * O.kernel_w(kernel, h, r), 0, h,
                              points=[h / 2], epsabs=1e-13, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-10


@pytest.mark.parametrize("kernel", KERNELS)
def test_kernel_support_and_positivity(kernel):
    h = 2.5
    assert O.kernel_w(kernel, h, h) == 0.0 and O.kernel_f(kernel, h, h) == 0.0
    assert O.kernel_w(kernel, h, 3.0) == 0.0
    r = np.linspace(0.0, h * 0.999, 301)
    assert all(O.kernel_w(kernel, h, x) > 0 for x in r)
    assert all(O.kernel_f(kernel, h, x) > 0 for x in r[1:])


@pytest.mark.parametrize("kernel", KERNELS)
def test_F_is_minus_Wprime_over_r(kernel):
    # grad W(r) = -F(|r|) r, i.e. F = -W'(r)/r (Sec. 2.1.1); pins reading A2
    h, d = 2.5, 1e-6
    for r in np.linspace(0.05, h - 0.05, 57):
        wp = (O.kernel_w(kernel, h, r + d) - O.kernel_w(kernel, h, r - d)) / (2 * d)
        assert abs(-wp / r - O.kernel_f(kernel, h, r)) < 1e-8


def test_cubic_matches_paper_formula_and_is_continuous():
    # eq. (sdpd-cubic-w) as printed, and continuity of W and F at h/2
    h = 2.5
    for r in [0.0, 0.3, 1.0, 1.25, 1.7, 2.2]:
        x = r / h
        w = 8 / (np.pi * h**3) * (1 - 6 * x**2 + 6 * x**3) if x <= 0.5 else \
            16 / (np.pi * h**3) * (1 - x)**3
        assert abs(O.kernel_w(O.KERNEL_CUBIC, h, r) - w) < 1e-15
    # first branch of F as printed by the paper
    for r in [0.1, 0.7, 1.2]:
        assert abs(O.kernel_f(O.KERNEL_CUBIC, h, r) - 48 / (np.pi * h**5) * (2 - 3 * r / h)) < 1e-15
    e = 1e-9
    for fn in (O.kernel_w, O.kernel_f):
        assert abs(fn(O.KERNEL_CUBIC, h, h / 2 - e) - fn(O.KERNEL_CUBIC, h, h / 2 + e)) < 1e-8


def test_kernel_self_values():
    # W(0): Lucy 105/(16 pi h^3), cubic 8/(pi h^3)
    h = 2.5
    assert abs(O.kernel_w(O.KERNEL_LUCY, h, 0.0) - 0.1336901522) < 1e-10
    assert abs(O.kernel_w(O.KERNEL_CUBIC, h, 0.0) - 0.1629746617) < 1e-10


def _params(**kw):
    base = dict(n=1, box=10.0, Cv=10.0, kB=1.0, m=1.0, rho0=1.0)
    base.update(kw)
    return O.OracleParams(**base)


@pytest.mark.parametrize("Cv,A,rho0", [(10.0, None, 1.0), (1.5, None, 0.7), (4.0, 2.5, 1.3)])
def test_closure_against_entropy_derivatives(Cv, A, rho0):
    # T = 1/dS/deps, P = -(rho^2/m) dS/drho / dS/deps, C = -(dS/deps)^2/d2S/deps2
    # (Sec. 2.1.2), by central differences of the oracle's S
    P = _params(Cv=Cv, A=A, rho0=rho0, m=1.7, kB=0.9)
    for eps, rho in [(10.0, 1.0), (0.15, 0.97), (3.3, 1.21)]:
        de, dr = 1e-5 * eps, 1e-5 * rho
        Se = (O.entropy(P, eps + de, rho) - O.entropy(P, eps - de, rho)) / (2 * de)
        See = (O.entropy(P, eps + de, rho) - 2 * O.entropy(P, eps, rho)
               + O.entropy(P, eps - de, rho)) / de**2
        Sr = (O.entropy(P, eps, rho + dr) - O.entropy(P, eps, rho - dr)) / (2 * dr)
        assert O.temperature(P, eps, rho) == pytest.approx(1 / Se, rel=1e-8)
        assert O.pressure(P, eps, rho) == pytest.approx(-(rho**2 / P.m) * Sr / Se, rel=1e-8)
        assert O.heat_capacity(P, eps, rho) == pytest.approx(-Se**2 / See, rel=1e-4)


def test_entropy_is_the_papers_ideal_gas():
    # eq. (pg-eos): S = (3/2)(K-1) kB ln eps - (1/2)(K-1) ln rho with kB restored
    # in the rho term (reading A4); compare differences (rho0 drops out)
    K = 5.0
    Cv = 1.5 * (K - 1.0)
    P = _params(Cv=Cv, rho0=2.0)

    def paper(eps, rho):
        return 1.5 * (K - 1) * np.log(eps) - 0.5 * (K - 1) * np.log(rho)

    for (e1, r1), (e2, r2) in [((1.0, 1.0), (2.0, 1.1)), ((0.3, 0.9), (7.0, 1.3))]:
        d_or = O.entropy(P, e1, r1) - O.entropy(P, e2, r2)
        assert d_or == pytest.approx(paper(e1, r1) - paper(e2, r2), rel=1e-13)
    # C = Cv = C_K of eq. (dist-analytic)
    assert O.heat_capacity(P, 0.7, 1.0) == pytest.approx(1.5 * (K - 1.0), rel=1e-14)


def test_constant_entropy_energy():
    # Sec. 3.1: eps = E(S, rho) inverts S at fixed rho
    P = _params(Cv=1.5)
    for eps, rho, rho2 in [(0.15, 1.0, 1.03), (10.0, 0.98, 0.95)]:
        S = O.entropy(P, eps, rho)
        e2 = O.eps_at_entropy(P, S, rho2)
        assert O.entropy(P, e2, rho2) == pytest.approx(S, abs=1e-12)
        assert O.eps_at_entropy(P, S, rho) == pytest.approx(eps, rel=1e-13)
