"""The Nc = 20 hard cases: mixtures within 2 % (in pressure) of a phase
boundary (bisection on the oracle's label, tests/hard_cases.py) and the
uniform Nc = 20 draw (z ~ Dirichlet(0.3), P up to 3e7 Pa): forward parity
against the oracle and the adjoint against the oracle's Jacobian; the
adjoint with one component set per mixture."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2205_03090_amd import _capi, api, workloads  # noqa: E402
from parity import assert_parity, compare, gpu_to_numpy, invariants  # noqa: E402
import hard_cases  # noqa: E402

pytestmark = pytest.mark.gpu
CLEAN = _capi.ST["INVALID"] | _capi.ST["SPLIT_UNCONV"] | _capi.ST["STEP_CAP"]


@pytest.fixture(scope="module")
def boundary():
    return hard_cases.boundary_workload(5, 300)


def _check_forward(w, tag, min_two_phase_frac, unconv_frac):
    r = api.flash(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij)
    torch.cuda.synchronize()
    g = gpu_to_numpy(r)
    inv = invariants(w, g)
    print(f"[{tag} invariants] {inv}", flush=True)
    assert inv["mass_balance"] < 1e-13 and inv["single_ok"] and inv["labels_valid"]
    o = oracle.flash(w, threads=8, want_min_tpd=1)
    rep = compare(g, o, w=w)
    print(f"[{tag}] {rep}", flush=True)
    # near the boundary the oracle's split stops unconverged on a few per
    # cent of the mixtures (checked there by equal fugacity instead)
    assert_parity(rep, o, path_agree=0.95, min_two_phase_frac=min_two_phase_frac,
                  unconv_frac=unconv_frac)
    return g


def test_boundary_nc20_forward_parity(boundary):
    print(f"case boundary nc=20 n={boundary.n}", flush=True)
    g = _check_forward(boundary, "boundary nc20", 0.3, 0.03)
    assert 0.2 < (g["label"] == 1).mean() < 0.8   # both sides of the boundary


def test_uniform_nc20_forward_parity():
    w = workloads.uniform_workload("c5_uniform", 2020, 2000, 20, 0.3, (200.0, 600.0),
                                   (1e5, 3e7))
    print(f"case uniform nc=20 n={w.n}", flush=True)
    _check_forward(w, "uniform nc20", 0.05, 0.005)


def _vjp_vs_oracle(w, idx_limit, seed, per_mixture=False):
    r = api.flash(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, keep_factor=True)
    gb, gx, gy = workloads.cotangents(seed, w.n, w.nc)
    gz, gT, gP, gk = api.flash_backward(w.z, w.T, w.P, w.Tc, w.Pc, w.omega, w.kij, r, gb, gx,
                                        gy, kij_reduce=False)
    torch.cuda.synchronize()
    gz, gT, gP, gk = (t.cpu().numpy() for t in (gz, gT, gP, gk))
    lab, beta, y = r.label.cpu().numpy(), r.beta.cpu().numpy(), r.y.cpu().numpy()
    st = r.status.cpu().numpy().astype(np.int64) & 0xffff
    two = np.where((lab == 1) & (st & CLEAN == 0) & (beta > 1e-3) & (beta < 1 - 1e-3))[0]
    two = two[:idx_limit]
    nc = w.nc
    pairs = [(a, b) for a in range(nc) for b in range(a + 1, nc)]
    worst = 0.0
    for m in two:
        sets = (w.Tc[m], w.Pc[m], w.omega[m], w.kij[m]) if per_mixture else \
            (w.Tc, w.Pc, w.omega, w.kij)
        ob = np.concatenate([[gb[m]], gx[m], gy[m]])
        args = (*sets, w.z[m], w.T[m], w.P[m], beta[m], y[m])
        # the reference at three finite-difference steps: their spread
        # estimates its own error (near a phase boundary the split is
        # ill-conditioned and the differences are far from converged)
        ref = oracle.flash_jacobian(*args, hrel=1e-3).T @ ob
        spread = max(np.abs(ref - oracle.flash_jacobian(*args, hrel=h).T @ ob).max()
                     for h in (3e-3, 3e-4))
        got = np.concatenate([gz[m], [gT[m], gP[m]],
                              [gk[m, a, b] + gk[m, b, a] for a, b in pairs]])
        tol = 1e-7 * np.abs(ref).max() + 10.0 * spread
        err = np.abs(got - ref).max() / tol
        worst = max(worst, err)
        assert err < 1.0, (m, np.abs(got - ref).max(), tol)
    return len(two), worst


def test_boundary_nc20_adjoint_vs_oracle_jacobian(boundary):
    print("case boundary nc=20 adjoint", flush=True)
    k, worst = _vjp_vs_oracle(boundary, 20, 9)
    print(f"[boundary nc20 adjoint] mixtures {k} worst error/tolerance {worst:.3f}", flush=True)
    assert k >= 10


def test_per_mixture_sets_adjoint_vs_oracle_jacobian():
    w = workloads.uniform_workload("pm_adj", 4040, 3000, 6, 0.5, (200.0, 600.0), (1e5, 2e7),
                                   per_mixture=True)
    print("case per-mixture sets nc=6 adjoint", flush=True)
    k, worst = _vjp_vs_oracle(w, 60, 13, per_mixture=True)
    print(f"[per-mixture adjoint] mixtures {k} worst error/tolerance {worst:.3f}", flush=True)
    assert k >= 40
