"""The flash's per-mixture work items (flash_stages.hpp, srk_device.hpp)
compiled for the host with g++ under the address and undefined-behaviour
sanitizers (tests/host_items), one mixture per thread, stages run to
completion in order as in the plain form.  Any out-of-bounds access, use of
freed memory, signed overflow, misaligned or null access, or non-finishing
item aborts the run; the results must also meet the parity bar against the
oracle (the host's exp/log round differently from the GPU's, so values are
compared with the oracle, not with the GPU).  Covers nc = 3, 8 and 20 with a
shared component set (nc = 20 reads its k table through the per-lane
pointer) and nc = 6 with one set per mixture; and nc = 20 once more under
the memory sanitizer, with the per-mixture records left unwritten, so that
a stage reading a record field no earlier stage wrote aborts the run."""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
from paper_2205_03090_amd import _capi, workloads
from host_items import runner
from parity import assert_parity, compare

CASES = {
    "nc3": lambda: workloads.nc3_workload(n=1000),
    "nc8": lambda: workloads.nc8_workload(n=1000, seed=77),
    "nc20": lambda: workloads.uniform_workload("p20", 920, 600, 20, 0.3, (200.0, 600.0),
                                               (1e5, 3e7)),
    "pm6": lambda: workloads.uniform_workload("pm6", 2006, 600, 6, 0.5, (200.0, 600.0),
                                              (1e5, 2e7), per_mixture=True),
}


@pytest.fixture(scope="module")
def built():
    # compile the per-nc executables in parallel (minutes on first use,
    # cached by source hash afterwards)
    jobs = [(3, "address"), (6, "address"), (8, "address"), (20, "address"), (20, "memory")]
    with cf.ThreadPoolExecutor(len(jobs)) as ex:
        list(ex.map(lambda j: runner.build(*j), jobs))
    o = _capi.default_options()
    return {f: getattr(o, f) for f, _ in o._fields_}


@pytest.mark.parametrize("case", sorted(CASES))
def test_host_items_sanitized_and_match_oracle(built, case):
    w = CASES[case]()
    g = runner.run(w, built, threads=4)
    o = oracle.flash(w, threads=4, want_min_tpd=1)
    rep = compare(g, o, w=w)
    print(f"[host {case}] {rep}")
    assert_parity(rep, o, path_agree=0.97, min_two_phase_frac=0.05)
    assert np.all((g["label"] == 0) | (g["label"] == 1))


def test_host_items_no_uninitialised_reads_nc20(built):
    w = workloads.uniform_workload("p20", 920, 300, 20, 0.3, (200.0, 600.0), (1e5, 3e7))
    g = runner.run(w, built, san="memory")
    o = oracle.flash(w, threads=4, want_min_tpd=1)
    rep = compare(g, o, w=w)
    print(f"[host msan nc20] {rep}")
    assert_parity(rep, o, path_agree=0.97, min_two_phase_frac=0.03)
