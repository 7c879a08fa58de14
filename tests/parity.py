"""Comparison of GPU flash results with the CPU oracle (shared by the GPU
tests, the smoke check and the benchmark's checks).

Rule: labels must be identical wherever the oracle's |min TPD| > 1e-9; where
both sides report two phases (outside the same band), beta, x and y agree
within 1e-10 absolute; where both report one phase, beta = -1 and
x = y = z/sum(z) bit for bit.  A two-phase row whose oracle split did not
converge (the oracle's SPLIT_UNCONV flag) has no reference values; when the
workload is given, the GPU's split there must instead satisfy equal
fugacities (max |ln y_i phi_i(y) - ln x_i phi_i(x)| < 1e-9, evaluated by the
oracle's phase model) and the material balance.  Where the Gibbs energy of
the split has several stationary points (liquid-liquid splits near a
three-phase region) the two sides' descent paths can end at different ones:
a two-phase row whose values differ is accepted when the GPU's split is
valid in the same sense and its Gibbs energy is not above the oracle's (the
equilibrium is the minimum of G); such rows are counted as alt_split.  A
valid GPU split at a different local minimum whose G is above the oracle's is
counted as alt_split_higher: the method (a descent from the substitution's
end point) reaches a local minimum, and where G has several, either side's
path can end in the higher one (on 400,000 mixtures of the hard-case Nc = 20
set, three rows had the higher minimum on the GPU's side and five on the
oracle's); assert_parity bounds their number.
"""
from __future__ import annotations

import numpy as np

TOL = 1e-10
BAND = 1e-9
FUG_TOL = 1e-9
ORC_SPLIT_UNCONV = 4


def _sets(w, m):
    return (w.Tc[m], w.Pc[m], w.omega[m], w.kij[m]) if w.per_mixture else \
        (w.Tc, w.Pc, w.omega, w.kij)


def split_gibbs(w, m: int, x, y, beta) -> float:
    """Reduced Gibbs energy per unit feed of the split (beta, x, y) of
    mixture m, sum over phases of phase fraction times sum c_i ln(c_i phi_i),
    with the oracle's phase model."""
    import oracle
    lx, _ = oracle.lnphi(*_sets(w, m), w.T[m], w.P[m], x)
    ly, _ = oracle.lnphi(*_sets(w, m), w.T[m], w.P[m], y)
    return float((1 - beta) * np.dot(x, np.log(x) + lx) + beta * np.dot(y, np.log(y) + ly))


def split_residual_max(w, m: int, x, y) -> float:
    """max_i |ln y_i + ln phi_i(y) - ln x_i - ln phi_i(x)| with the oracle's
    phase model, for mixture m of workload w."""
    import oracle
    lx, _ = oracle.lnphi(*_sets(w, m), w.T[m], w.P[m], x)
    ly, _ = oracle.lnphi(*_sets(w, m), w.T[m], w.P[m], y)
    return float(np.abs(np.log(y) + ly - np.log(x) - lx).max())


def gpu_to_numpy(r):
    out = {k: getattr(r, k).detach().cpu().numpy() for k in
           ("label", "beta", "x", "y", "iters", "status", "flops")}
    if r.factor is not None:
        out["factor"] = r.factor.detach().cpu().numpy()
    if getattr(r, "tm", None) is not None:
        out["tm"] = r.tm.detach().cpu().numpy()
    return out


def compare(g: dict, o: dict, idx=None, verbose: bool = True, w=None) -> dict:
    """g: GPU arrays (full batch); o: oracle arrays for rows idx (or all);
    w: the workload of the full batch (enables the checks of rows whose
    oracle split did not converge)."""
    if idx is None:
        idx = np.arange(len(o["label"]))
    gl, ol = g["label"][idx].astype(int), o["label"].astype(int)
    mt = o["min_tpd"]
    decisive = ~(np.abs(mt) <= BAND)          # NaN (not computed) counts as decisive
    lab_bad = np.where(decisive & (gl != ol))[0]
    # values are compared where both report two phases outside the band
    # (within it G is flat to ~1e-9 and distinct stationary points compete)
    # and the oracle's split converged
    ref_unconv = (o["info"][:, 8] & ORC_SPLIT_UNCONV) != 0
    unc2 = np.where((gl == 1) & (ol == 1) & decisive & ref_unconv)[0]
    both2 = np.where((gl == 1) & (ol == 1) & decisive & ~ref_unconv)[0]
    both1 = np.where((gl == 0) & (ol == 0))[0]
    db = np.abs(g["beta"][idx][both2] - o["beta"][both2]) if len(both2) else np.zeros(0)
    dx = np.abs(g["x"][idx][both2] - o["x"][both2]).max(1) if len(both2) else np.zeros(0)
    dy = np.abs(g["y"][idx][both2] - o["y"][both2]).max(1) if len(both2) else np.zeros(0)
    err = np.maximum(db, np.maximum(dx, dy))
    val_bad = both2[err > TOL]
    # a different valid split: with Gibbs energy not above the oracle's, or
    # at another local minimum above it
    alt, alt_hi = [], []
    if w is not None and len(val_bad):
        keep = []
        for k in val_bad:
            m = idx[k]
            xr, yr, b = g["x"][m], g["y"][m], g["beta"][m]
            zz = w.z[m] / np.cumsum(w.z[m])[-1]
            valid = split_residual_max(w, m, xr, yr) < FUG_TOL and \
                float(np.abs((1 - b) * xr + b * yr - zz).max()) < 1e-13
            Gg = split_gibbs(w, m, xr, yr, b)
            Go = split_gibbs(w, m, o["x"][k], o["y"][k], o["beta"][k])
            if valid and Gg <= Go + 1e-12 * max(1.0, abs(Go)):
                alt.append(k)
            elif valid:
                alt_hi.append(k)
                if verbose:
                    print(f"  row {m}: another local minimum of G, {Gg - Go:+.3e} above the "
                          f"oracle's (gpu beta {b:.12g}, oracle beta {o['beta'][k]:.12g})",
                          flush=True)
            else:
                keep.append(k)
        val_bad = np.asarray(keep, dtype=both2.dtype)
    if len(alt) or len(alt_hi):
        err = err.copy()
        err[np.searchsorted(both2, alt + alt_hi)] = 0.0
    one_bad = both1[(g["beta"][idx][both1] != -1.0) |
                    np.any(g["x"][idx][both1] != o["x"][both1], axis=1) |
                    np.any(g["y"][idx][both1] != o["y"][both1], axis=1)]
    # rows without a converged reference: the GPU split must be valid
    unc_bad, unc_res = [], 0.0
    if w is not None:
        for k in unc2:
            m = idx[k]
            xr, yr, b = g["x"][m], g["y"][m], g["beta"][m]
            zz = w.z[m] / np.cumsum(w.z[m])[-1]
            res = split_residual_max(w, m, xr, yr)
            mb = float(np.abs((1 - b) * xr + b * yr - zz).max())
            unc_res = max(unc_res, res)
            if not (res < FUG_TOL and mb < 1e-13):
                unc_bad.append(k)
    else:
        unc_bad = list(unc2)
    val_bad = np.concatenate([val_bad, np.asarray(unc_bad, dtype=val_bad.dtype)])
    rep = dict(n=len(idx), two_phase=int(len(both2)), single=int(len(both1)),
               label_mismatch=int(len(lab_bad)), value_mismatch=int(len(val_bad)),
               single_mismatch=int(len(one_bad)),
               max_err=float(err.max()) if len(err) else 0.0,
               band_excluded=int((~decisive).sum()),
               ref_unconverged=int(len(unc2)), ref_unconverged_residual=unc_res,
               alt_split=int(len(alt)), alt_split_higher=int(len(alt_hi)))
    # path agreement of the substitution counters (same algorithm on both sides)
    oi, gi = o["info"], g["iters"][idx]
    same = (gi[:, 0] == oi[:, 1]) & (gi[:, 1] == oi[:, 2]) & (gi[:, 3] == oi[:, 4]) & \
           (gi[:, 5] == oi[:, 6])
    rep["ss_path_agree"] = float(same.mean()) if len(same) else 1.0
    if verbose and (len(lab_bad) or len(val_bad) or len(one_bad)):
        for k in list(lab_bad[:5]) + list(val_bad[:5]) + list(one_bad[:3]):
            m = idx[k]
            print(f"  row {m}: gpu label {gl[k]} beta {g['beta'][m]:.12g} iters "
                  f"{g['iters'][m].tolist()} status {int(g['status'][m]) & 0xffff:#x} | oracle "
                  f"label {ol[k]} beta {o['beta'][k]:.12g} min_tpd {mt[k]:.3e} info "
                  f"{o['info'][k].tolist()} | err {err[np.searchsorted(both2, k)] if k in both2 else 0:.2e}",
                  flush=True)
    return rep


def invariants(w, g) -> dict:
    """Checks every GPU output: material balance and normalisation of
    two-phase results; single-phase results equal the normalised feed."""
    lab = g["label"]
    two = lab == 1
    z = w.z / np.cumsum(w.z, axis=1)[:, -1:]
    b = g["beta"][two][:, None]
    mb = np.abs((1 - b) * g["x"][two] + b * g["y"][two] - z[two]).max() if two.any() else 0.0
    sx = np.abs(g["x"][two].sum(1) - 1).max() if two.any() else 0.0
    sy = np.abs(g["y"][two].sum(1) - 1).max() if two.any() else 0.0
    brange = bool(np.all((g["beta"][two] > 0) & (g["beta"][two] < 1)))
    one = lab == 0
    single_ok = bool(np.all(g["beta"][one] == -1.0) and np.array_equal(g["x"][one], z[one])
                     and np.array_equal(g["y"][one], z[one]))
    return dict(two_phase_frac=float(two.mean()), mass_balance=float(mb), sum_x=float(sx),
                sum_y=float(sy), beta_in_range=brange, single_ok=single_ok,
                labels_valid=bool(np.all((lab == 0) | (lab == 1))))


def assert_parity(rep: dict, o: dict | None = None, path_agree: float = 0.97,
                  min_two_phase_frac: float = 0.05, alt_frac: float = 0.01,
                  unconv_frac: float = 0.005, alt_higher_frac: float = 0.002) -> None:
    """The parity bar plus guards that keep it from passing vacuously: no
    label, value or single-phase mismatch; at most 1 % of the rows inside
    the min-TPD band (at least one row allowed below 100 rows); at most
    unconv_frac of the rows without a converged oracle split, alt_frac of
    the compared two-phase rows on a second valid split and alt_higher_frac
    (at least one row) at a local minimum above the oracle's; and a floor on the
    two-phase rows whose values were compared: at least 90 % of the oracle's
    two-phase rows, which in turn are at least min_two_phase_frac of the
    rows."""
    n = rep["n"]
    assert rep["label_mismatch"] == 0, rep
    assert rep["value_mismatch"] == 0, rep
    assert rep["single_mismatch"] == 0, rep
    assert rep["ss_path_agree"] >= path_agree, rep
    assert rep["band_excluded"] <= max(0.01 * n, 1 if n < 100 else 0), rep
    assert rep["ref_unconverged"] <= unconv_frac * n, rep
    assert rep["alt_split"] <= alt_frac * max(1, rep["two_phase"]), rep
    assert rep["alt_split_higher"] <= max(1, alt_higher_frac * rep["two_phase"]), rep
    if o is not None:
        o2 = int((np.asarray(o["label"]) == 1).sum())
        assert o2 >= min_two_phase_frac * n, (o2, rep)
        assert rep["two_phase"] >= 0.9 * o2, (o2, rep)
    else:
        assert rep["two_phase"] >= min_two_phase_frac * n, rep
