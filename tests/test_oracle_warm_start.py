"""Pins of the oracle's warm-start inputs (Sec. 4: where a classifier's
label and an initializer's K enter the flash): an initial ln K in place of
Wilson's and a per-mixture stable/unstable hint.

What fixes the expected values here is not the oracle itself:
* an initial ln K equal to Wilson's (computed by the oracle's separate Wilson
  probe) must reproduce the un-hinted flash bit for bit;
* hint values other than 0 and 1 mean "no hint": bit for bit the same flash;
* a mixture hinted stable is the normalised feed, untouched;
* the equilibrium of a two-phase mixture does not depend on where the split
  starts, within its basin (the minimum of G is unique away from
  three-phase regions): a hinted-unstable flash from Wilson's K where they
  carried the plain flash's triage, and one from the converged K of a
  previous flash, reach the same beta, x, y within the split's tolerance,
  and the latter converges in fewer substitutions; where Wilson's K admit
  no split the hinted split is reported failed, and submitting it again
  without the hint gives the plain result;
* a non-finite initial ln K is invalid input.
"""
import numpy as np
import pytest

from paper_2205_03090_amd import workloads


def _fields(orc):
    return {k: i for i, k in enumerate(orc.INFO_FIELDS)}


@pytest.fixture(scope="module")
def w8():
    return workloads.uniform_workload("ws8", 5150, 1000, 8, 0.5, (200.0, 600.0), (1e5, 2e7))


@pytest.fixture(scope="module")
def base(orc, w8):
    return orc.flash(w8, threads=8)


def _wilson(orc, w):
    return np.stack([orc.wilson_lnk(w.Tc, w.Pc, w.omega, w.T[m], w.P[m]) for m in range(w.n)])


def _same(a, b):
    for k in ("label", "beta", "x", "y", "info"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert np.array_equal(a["tm"], b["tm"], equal_nan=True)


def test_wilson_lnk0_reproduces_the_plain_flash(orc, w8, base):
    r = orc.flash(w8, threads=8, lnk0=_wilson(orc, w8))
    _same(r, base)


def test_no_hint_values(orc, w8, base):
    rng = np.random.Generator(np.random.PCG64(3))
    hint = rng.choice(np.array([-1, 2, 7, -128], dtype=np.int8), w8.n)
    _same(orc.flash(w8, threads=8, hint=hint), base)


def test_hint_stable_is_the_feed(orc, w8, base):
    F = _fields(orc)
    hint = np.zeros(w8.n, np.int8)
    r = orc.flash(w8, threads=8, hint=hint)
    z = w8.z / w8.z.sum(1, keepdims=True)
    assert np.all(r["label"] == 0)
    assert np.all(r["beta"] == -1.0)
    assert np.allclose(r["x"], z, rtol=0, atol=1e-15) and np.array_equal(r["x"], r["y"])
    assert np.all(r["info"][:, F["flags"]] == orc.FLAG_HINTED)
    assert np.all(r["info"][:, F["case"]] == 0) and np.all(np.isnan(r["tm"]))
    # the stable rows of the plain flash are the same feed
    one = base["label"] == 0
    assert np.array_equal(r["x"][one], base["x"][one])


def _two_phase_converged(orc, r):
    F = _fields(orc)
    return (r["label"] == 1) & ((r["info"][:, F["flags"]] & orc.FLAG_SPLIT_UNCONV) == 0)


def test_hint_unstable_reaches_the_same_split(orc, w8, base):
    F = _fields(orc)
    two = _two_phase_converged(orc, base)
    assert two.sum() > 120
    hint = np.where(base["label"] == 1, 1, -1).astype(np.int8)
    r = orc.flash(w8, threads=8, hint=hint)
    assert np.all(r["info"][two, F["case"]] == 4)
    assert np.all(r["info"][two, F["flags"]] & orc.FLAG_HINTED)
    assert np.all(r["info"][two, F["ss_v"]] == 0) and np.all(r["info"][two, F["pre"]] == 0)
    assert np.all(np.isnan(r["tm"][two]))
    # where Wilson's K carries the split (the triage of the plain flash found
    # the instability from them: case 3) the hinted split ends at the same
    # equilibrium
    c3 = two & (base["info"][:, F["case"]] == 3)
    assert c3.sum() > 50
    ok = c3 & _two_phase_converged(orc, r)
    assert ok.sum() > 0.97 * c3.sum()
    db = np.abs(r["beta"][ok] - base["beta"][ok])
    dx = np.abs(r["x"][ok] - base["x"][ok]).max(1)
    dy = np.abs(r["y"][ok] - base["y"][ok]).max(1)
    same = np.maximum(db, np.maximum(dx, dy)) < 1e-10
    assert same.mean() > 0.97, same.mean()
    # where Wilson's K put every K on one side of 1 or theta outside (0, 1)
    # (case 1), the split from them fails and says so: single phase with
    # SPLIT_FAILED, so that the caller can submit those mixtures again
    # without the hint, which gives the plain flash's result
    failed = (r["info"][:, F["flags"]] & orc.FLAG_SPLIT_FAILED) != 0
    assert np.all(r["label"][failed] == 0)
    assert np.all(base["info"][failed & two, F["case"]] == 1)
    idx = np.where(failed)[0]
    assert len(idx) > 0
    again = orc.flash(w8.subset(idx), threads=8)
    for k in ("label", "beta", "x", "y", "info"):
        assert np.array_equal(again[k], base[k][idx], equal_nan=True), k
    # un-hinted rows are untouched
    rest = hint == -1
    for k in ("label", "beta", "x", "y", "info"):
        assert np.array_equal(r[k][rest], base[k][rest], equal_nan=True), k


def test_warm_start_from_a_previous_result(orc, w8, base):
    # the converged K of a previous step (a time step of a simulator, or a
    # re-submitted mixture) as the initial K: the same split, found sooner
    F = _fields(orc)
    two = _two_phase_converged(orc, base)
    lnk0 = _wilson(orc, w8)
    lnk0[two] = np.log(base["y"][two] / base["x"][two])
    hint = np.where(two, 1, -1).astype(np.int8)
    r = orc.flash(w8, threads=8, lnk0=lnk0, hint=hint)
    assert np.all(r["label"][two] == 1)
    err = np.maximum(np.abs(r["beta"][two] - base["beta"][two]),
                     np.maximum(np.abs(r["x"][two] - base["x"][two]).max(1),
                                np.abs(r["y"][two] - base["y"][two]).max(1)))
    assert err.max() < 1e-10
    ss_w = r["info"][two, F["ss_split"]]
    ss_b = base["info"][two, F["ss_split"]] + base["info"][two, F["pre"]]
    assert ss_w.mean() < 0.5 * ss_b.mean()
    assert ss_w.max() <= 2
    assert np.all(r["info"][two, F["nt_split"]] <= 2)


def test_non_finite_lnk0_is_invalid(orc, w8):
    F = _fields(orc)
    lnk0 = _wilson(orc, w8)[:50].copy()
    lnk0[3, 2] = np.nan
    lnk0[7, 0] = np.inf
    sub = w8.subset(np.arange(50))
    r = orc.flash(sub, lnk0=lnk0)
    bad = r["info"][:, F["flags"]] & orc.FLAG_INVALID
    assert bad[3] and bad[7] and bad.sum() == 2
