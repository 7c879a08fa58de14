"""Pins of the oracle's equation-of-state layer (SRK, Appendix A).

Each test checks the oracle against something other than its own formulas:
numpy's polynomial roots, the thermodynamic definition of the fugacity
coefficient (integral of (Z-1)/P and the partial molar derivative of n*g_res),
Soave's acentric-factor construction, the SRK critical point and the
ideal-gas limit.
"""
import numpy as np
import pytest


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_cubic_roots_match_numpy(orc):
    rng = _rng(1)
    n3 = 0
    for _ in range(3000):
        A = 10 ** rng.uniform(-4, 1.3)
        B = 10 ** rng.uniform(-5, -0.3)
        got = orc.cubic_roots(A, B)
        r1, r0 = A - B * (1 + B), A * B
        ref = np.roots([1.0, -1.0, r1, -r0])
        ref = np.sort(ref[np.abs(ref.imag) < 1e-9 * np.abs(ref)].real)
        ref = ref[ref > B]
        if len(ref) != len(got):
            # only at a near-double root may the counts legitimately differ
            f = lambda Z: ((Z - 1) * Z + r1) * Z - r0
            zs = (1 + np.sqrt(max(1 - 3 * r1, 0)) * np.array([-1, 1])) / 3
            assert min(abs(f(zs))) < 1e-10
            continue
        assert np.allclose(got, ref, rtol=1e-9, atol=1e-12)
        if len(got) == 3:
            n3 += 1
            # Vieta: sum = 1, pair sum = rho1, product = rho0
            assert abs(got.sum() - 1.0) < 1e-12
            assert abs(got[0] * got[1] + got[0] * got[2] + got[1] * got[2] - r1) < 1e-12
            assert abs(got.prod() - r0) < 1e-12 * max(1.0, r0)
    assert n3 > 100


def test_cubic_root_is_bracketed_and_signchange(orc):
    # every reported root is a sign change of f to within adjacent doubles
    rng = _rng(2)
    for _ in range(500):
        A, B = 10 ** rng.uniform(-3, 1), 10 ** rng.uniform(-4, -0.5)
        r1, r0 = A - B * (1 + B), A * B
        f = lambda Z: ((Z - 1) * Z + r1) * Z - r0
        for Z in orc.cubic_roots(A, B):
            assert B < Z < 1 + B
            lo, hi = np.nextafter(Z, -np.inf), np.nextafter(Z, np.inf)
            for _ in range(3):
                lo, hi = np.nextafter(lo, -np.inf), np.nextafter(hi, np.inf)
            assert f(lo) * f(hi) <= 0 or abs(f(Z)) < 1e-15


def test_srk_critical_point_triple_root(orc):
    # At T = Tc, P = Pc a pure SRK fluid has (up to the rounded Omega
    # constants) a triple root Z = 1/3; the rounded constants perturb the
    # coefficients by ~1e-6, i.e. the root by ~(1e-6)^(1/3).
    lp, info = orc.lnphi([400.0], [4e6], [0.2], [[0.0]], 400.0, 4e6, [1.0])
    assert abs(info["A"] - 1 / 3 - info["B"] - info["B"] ** 2) < 1e-5
    assert abs(info["A"] * info["B"] - 1 / 27) < 1e-6
    assert abs(info["Z"] - 1 / 3) < 0.02


def _pure_psat(orc, Tc, Pc, om, T):
    lo, hi = 1e2, 0.999 * Pc
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        Z = orc.lnphi([Tc], [Pc], [om], [[0.0]], T, mid, [1.0])[1]["Z"]
        if Z > 0.3:
            lo = mid
        else:
            hi = mid
    return lo, hi


@pytest.mark.parametrize("om", [0.0, 0.05, 0.15, 0.3, 0.45])
def test_soave_acentric_factor_construction(orc, om):
    # Soave fitted m(omega) so that SRK reproduces the definition of the
    # acentric factor: log10(Psat/Pc) = -1 - omega at T = 0.7 Tc.  This pins
    # Omega_a, Omega_b, alpha(T), m(omega), the min-Gibbs root choice and ln phi
    # together (the chosen root jumps from vapour to liquid at Psat).
    Tc, Pc = 400.0, 4.0e6
    lo, hi = _pure_psat(orc, Tc, Pc, om, 0.7 * Tc)
    assert abs(np.log10(0.5 * (lo + hi) / Pc) + 1 + om) < 2e-3
    # equal fugacity of the two roots at Psat
    a = orc.lnphi([Tc], [Pc], [om], [[0.0]], 0.7 * Tc, lo, [1.0])
    b = orc.lnphi([Tc], [Pc], [om], [[0.0]], 0.7 * Tc, hi, [1.0])
    assert a[1]["nroots"] == 3 and b[1]["nroots"] == 3
    assert abs(a[0][0] - b[0][0]) < 1e-9


def test_ideal_gas_limit(orc):
    rng = _rng(3)
    for _ in range(20):
        nc = 5
        Tc, Pc, om = rng.uniform(190, 620, nc), rng.uniform(2e6, 5e6, nc), rng.uniform(0.01, 0.5, nc)
        k = np.zeros((nc, nc))
        c = rng.dirichlet(np.ones(nc))
        lp, info = orc.lnphi(Tc, Pc, om, k, 400.0, 1e-2, c)
        assert np.abs(lp).max() < 1e-8
        assert abs(info["Z"] - 1) < 1e-8


def _sample_mixture(rng, nc):
    Tc, Pc, om = rng.uniform(190, 620, nc), rng.uniform(2e6, 5e6, nc), rng.uniform(0.01, 0.5, nc)
    k = np.zeros((nc, nc))
    iu = np.triu_indices(nc, 1)
    k[iu] = rng.uniform(0, 0.15, len(iu[0]))
    return Tc, Pc, om, k + k.T


def test_gres_is_integral_of_compressibility(orc):
    # ln phi of the mixture (= g_res) is the integral over pressure of
    # (Z - 1)/P at fixed T and composition.  Cases are supercritical-like
    # (high T), where a single root persists along the path.
    rng = _rng(4)
    for _ in range(6):
        nc = 4
        Tc, Pc, om, k = _sample_mixture(rng, nc)
        T = 1.6 * Tc.max()
        P = rng.uniform(2e6, 1.5e7)
        c = rng.dirichlet(np.ones(nc))
        # integrate in ln P: int (Z-1) dlnP from ~0 to P (Gauss-Legendre)
        xs, ws = np.polynomial.legendre.leggauss(200)
        lo, hi = np.log(1e-3), np.log(P)
        u = 0.5 * (hi - lo) * xs + 0.5 * (hi + lo)
        Zs = np.array([orc.lnphi(Tc, Pc, om, k, T, np.exp(v), c)[1]["Z"] for v in u])
        for v in u:
            assert orc.lnphi(Tc, Pc, om, k, T, np.exp(v), c)[1]["nroots"] == 1
        integral = 0.5 * (hi - lo) * np.sum(ws * (Zs - 1.0))
        lp, info = orc.lnphi(Tc, Pc, om, k, T, P, c)
        assert abs(np.dot(c, lp) - integral) < 1e-9
        assert abs(orc.gres(info["Z"], info["A"], info["B"]) - integral) < 1e-9


def test_lnphi_is_partial_molar_gres(orc):
    # ln phi_i = d(n g_res)/d n_i at fixed T, P (central differences of
    # n * g_res(Z, A, B) with A, B, Z taken from the EOS at each composition).
    rng = _rng(5)
    for trial in range(30):
        nc = int(rng.integers(2, 9))
        Tc, Pc, om, k = _sample_mixture(rng, nc)
        T, P = rng.uniform(200, 600), rng.uniform(1e5, 2e7)
        n = rng.dirichlet(np.ones(nc)) * 2.0
        lp, info = orc.lnphi(Tc, Pc, om, k, T, P, n / n.sum())

        def ng(nn):
            _, inf = orc.lnphi(Tc, Pc, om, k, T, P, nn / nn.sum())
            return nn.sum() * orc.gres(inf["Z"], inf["A"], inf["B"]), inf
        _, base = ng(n)
        for i in range(nc):
            h = 1e-5 * n[i]
            e = np.zeros(nc); e[i] = h
            fp, ip = ng(n + e)
            fm, im = ng(n - e)
            if abs(ip["Z"] - base["Z"]) > 1e-3 or abs(im["Z"] - base["Z"]) > 1e-3:
                continue  # root switch inside the stencil
            d = (fp - fm) / (2 * h)
            assert abs(d - lp[i]) < 1e-6 * max(1.0, abs(lp[i])), (trial, i, d, lp[i])


def test_min_gibbs_root_choice(orc):
    # Where three roots exist, the chosen root has the lower g_res.
    rng = _rng(6)
    seen = 0
    for _ in range(3000):
        nc = 3
        Tc, Pc, om, k = _sample_mixture(rng, nc)
        T, P = rng.uniform(200, 600), rng.uniform(1e5, 2e7)
        c = rng.dirichlet(np.ones(nc))
        _, info = orc.lnphi(Tc, Pc, om, k, T, P, c)
        if info["nroots"] == 3:
            seen += 1
            g = [orc.gres(Z, info["A"], info["B"]) for Z in info["roots"][[0, 2]]]
            assert info["Z"] == info["roots"][int(np.argmin(g)) * 2]
    assert seen > 20


def test_wilson_reproduces_acentric_definition(orc):
    # The Wilson constant 5.373 ~= (7/3) ln 10: at T = 0.7 Tc and
    # P = Pc 10^(-1-omega) (the acentric-factor point), K = 1.
    for om in (0.0, 0.2, 0.5):
        lnK = orc.wilson_lnk([400.0], [4e6], [om], 280.0, 4e6 * 10 ** (-1 - om))
        assert abs(lnK[0]) < 5e-4
    lnK = orc.wilson_lnk([300.0, 500.0], [4e6, 3e6], [0.1, 0.3], 300.0, 4e6)
    assert abs(lnK[0]) < 1e-15  # T = Tc and P = Pc give K = 1


def test_tpd_ideal_gas_is_kl_divergence(orc):
    # At vanishing pressure ln phi -> 0 and tpd(w) = sum w ln(w/z) >= 0.
    rng = _rng(7)
    for _ in range(20):
        nc = 4
        Tc, Pc, om, k = _sample_mixture(rng, nc)
        z, w = rng.dirichlet(np.ones(nc)), rng.dirichlet(np.ones(nc))
        t = orc.tpd(Tc, Pc, om, k, 400.0, 1e-2, z, w)
        assert abs(t - np.sum(w * np.log(w / z))) < 1e-9
        assert abs(orc.tpd(Tc, Pc, om, k, 300.0, 5e6, z, z)) < 1e-13


def test_kij_combining_rule_identical_components(orc):
    # Two components with the same Tc, Pc and omega differ only through
    # k_12 = k in the combining rule (Appendix A, eq. mixing_rule:
    # (a alpha)_ij = (1 - k_ij) sqrt(a_i alpha_i a_j alpha_j)).  Then
    #   A_mix = A_0 (c1^2 + c2^2 + 2 (1 - k) c1 c2) = A_0 (1 - 2 k c1 c2),
    #   psi_1 - psi_2 = A_0 k (c1 - c2), and from eq. lnphi
    #   ln phi_1 - ln phi_2 = -(2 A_0 k / B) ln(1 + B/Z) (c1 - c2),
    # with A_0 the pure-component value (any composition at k = 0) and B
    # composition-independent.  A sign error (1 + k), a doubled k or a
    # transposed index in the combining rule fails one of the two identities.
    rng = _rng(41)
    for _ in range(200):
        tc, pc, om = rng.uniform(190, 620), rng.uniform(2e6, 5e6), rng.uniform(0.01, 0.5)
        Tc, Pc, omega = np.array([tc, tc]), np.array([pc, pc]), np.array([om, om])
        k = rng.uniform(0.0, 0.3)
        kij = np.array([[0.0, k], [k, 0.0]])
        T, P = rng.uniform(200, 600), rng.uniform(1e5, 2e7)
        c = rng.dirichlet([1, 1])
        _, i0 = orc.lnphi(Tc, Pc, omega, np.zeros((2, 2)), T, P, c)
        lp, info = orc.lnphi(Tc, Pc, omega, kij, T, P, c)
        A0, A, B, Z = i0["A"], info["A"], info["B"], info["Z"]
        assert abs(info["B"] - i0["B"]) <= 1e-15 * i0["B"]
        assert abs(A - A0 * (1.0 - 2.0 * k * c[0] * c[1])) <= 1e-14 * A0
        ref = -(2.0 * A0 * k / B) * np.log1p(B / Z) * (c[0] - c[1])
        assert abs((lp[0] - lp[1]) - ref) <= 1e-12 * max(1.0, abs(ref))


def test_kij_enters_symmetric_pairs_only(orc):
    # A ternary with k_12 = k_21 = k and the rest zero: exchanging the
    # compositions of components 1 and 2 (identical pure properties for 1
    # and 2) leaves A unchanged and exchanges ln phi_1 and ln phi_2, while
    # component 3 (not in the pair) keeps its ln phi; with k = 0 the value of
    # A is the square of sum_i c_i sqrt(A_i).
    rng = _rng(42)
    for _ in range(100):
        tc, pc, om = rng.uniform(190, 620), rng.uniform(2e6, 5e6), rng.uniform(0.01, 0.5)
        Tc = np.array([tc, tc, rng.uniform(190, 620)])
        Pc = np.array([pc, pc, rng.uniform(2e6, 5e6)])
        omega = np.array([om, om, rng.uniform(0.01, 0.5)])
        k = rng.uniform(0.0, 0.15)
        kij = np.zeros((3, 3))
        kij[0, 1] = kij[1, 0] = k
        T, P = rng.uniform(200, 600), rng.uniform(1e5, 2e7)
        c = rng.dirichlet([1, 1, 1])
        cs = c[[1, 0, 2]]
        l1, i1 = orc.lnphi(Tc, Pc, omega, kij, T, P, c)
        l2, i2 = orc.lnphi(Tc, Pc, omega, kij, T, P, cs)
        assert abs(i1["A"] - i2["A"]) <= 1e-14 * i1["A"]
        if i1["Z"] == i2["Z"]:
            assert np.allclose(l1[[1, 0, 2]], l2, rtol=0, atol=1e-12)
        # k = 0: A = (sum c_i sqrt(A_i))^2 with A_i the pure values
        _, i0 = orc.lnphi(Tc, Pc, omega, np.zeros((3, 3)), T, P, c)
        Ai = []
        for j in range(3):
            e = np.full(3, 1e-300)
            e[j] = 1.0
            Ai.append(orc.lnphi(Tc, Pc, omega, np.zeros((3, 3)), T, P, e)[1]["A"])
        assert abs(i0["A"] - np.dot(c, np.sqrt(Ai)) ** 2) <= 1e-13 * i0["A"]
