"""Pins of the oracle's implicit-function Jacobian of the converged split:
against central differences of the full oracle flash (re-solved at p +- h,
h = 1e-6 relative), the identities that follow from the material balance and
normalisation, and the binary tie-line invariance (dx/dz = dy/dz = 0)."""
import numpy as np

from paper_2205_03090_amd import workloads
from paper_tables import components


def _flash_vec(orc, w, z, T, P, k):
    ww = workloads.Workload("x", 1, w.nc, z[None], np.array([T]), np.array([P]), w.Tc, w.Pc,
                            w.omega, k)
    r = orc.flash(ww)
    return r["label"][0], np.concatenate([[r["beta"][0]], r["x"][0], r["y"][0]])


def test_jacobian_matches_full_flash_differences(orc):
    w = workloads.nc3_workload(n=2000)
    r = orc.flash(w, threads=8)
    two = np.where((r["label"] == 1) & (r["beta"] > 1e-2) & (r["beta"] < 0.99))[0][:8]
    nc = w.nc
    pairs = [(a, b) for a in range(nc) for b in range(a + 1, nc)]
    for m in two:
        z, T, P = w.z[m], w.T[m], w.P[m]
        J = orc.flash_jacobian(w.Tc, w.Pc, w.omega, w.kij, z, T, P, r["beta"][m], r["y"][m])
        for q in range(J.shape[1]):
            dz = np.zeros(nc); dT = dP = 0.0; dk = np.zeros((nc, nc))
            if q < nc:
                h = 1e-6 * z[q]; dz[q] = h
            elif q == nc:
                h = 1e-6 * T; dT = h
            elif q == nc + 1:
                h = 1e-6 * P; dP = h
            else:
                h = 1e-6; a, b = pairs[q - nc - 2]; dk[a, b] = dk[b, a] = h
            lp, fp = _flash_vec(orc, w, z + dz, T + dT, P + dP, w.kij + dk)
            lm, fm = _flash_vec(orc, w, z - dz, T - dT, P - dP, w.kij - dk)
            assert lp == 1 and lm == 1
            fd = (fp - fm) / (2 * h)
            assert np.abs(fd - J[:, q]).max() < 1e-5 * max(1.0, np.abs(J).max()), (m, q)


def test_jacobian_identities(orc):
    w = workloads.nc8_workload(n=3000, seed=12)
    r = orc.flash(w, threads=8)
    two = np.where((r["label"] == 1) & (r["beta"] > 1e-3) & (r["beta"] < 1 - 1e-3))[0][:20]
    nc = w.nc
    for m in two:
        z = w.z[m]
        J = orc.flash_jacobian(w.Tc, w.Pc, w.omega, w.kij, z, w.T[m], w.P[m], r["beta"][m],
                               r["y"][m])
        scale = np.abs(J).max()
        db, dx, dy = J[0], J[1:1 + nc], J[1 + nc:]
        # sum x = sum y = 1
        assert np.abs(dx.sum(0)).max() < 1e-7 * scale
        assert np.abs(dy.sum(0)).max() < 1e-7 * scale
        # (1-beta) x + beta y = z/sum z, differentiated
        b, x, y = r["beta"][m], r["x"][m], r["y"][m]
        lhs = (1 - b) * dx + b * dy + np.outer(y - x, db)
        s = z.sum()
        rhs = np.zeros_like(lhs)
        rhs[:, :nc] = (np.eye(nc) - np.outer(z / s, np.ones(nc))) / s
        assert np.abs(lhs - rhs).max() < 1e-6 * scale
        # outputs are homogeneous of degree 0 in z
        assert np.abs(J[:, :nc] @ z).max() < 1e-6 * scale


def test_binary_jacobian_tie_line(orc):
    Tc, Pc, om, k = components(["CH4", "C6H14"])
    rng = np.random.Generator(np.random.PCG64(4))
    done = 0
    for _ in range(200):
        z = rng.dirichlet([1, 1]); T = rng.uniform(200, 500); P = rng.uniform(1e5, 1e7)
        w = workloads.Workload("b", 1, 2, z[None], np.array([T]), np.array([P]), Tc, Pc, om, k)
        r = orc.flash(w)
        if r["label"][0] != 1 or not (1e-3 < r["beta"][0] < 1 - 1e-3):
            continue
        J = orc.flash_jacobian(Tc, Pc, om, k, z, T, P, r["beta"][0], r["y"][0])
        assert np.abs(J[1:, :2]).max() < 1e-6 * max(1.0, np.abs(J).max())
        done += 1
    assert done > 10
