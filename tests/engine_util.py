"""Helpers that drive the HIP engine through its C ABI for the tests."""
import numpy as np

import paper_2603_26576_amd as hp


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def new_session(trace, device=False, tuning=None):
    s = hp.hpop_session_create(trace.n_hosts, trace.n_devices)
    if tuning:
        hp.hpop_session_set_tuning(s, **tuning)
    chunks = [(c.resource, c.kind, c.start, c.end) for c in trace.chunks]
    keep = hp.add_chunks(s, chunks, device=device) if chunks else []
    for t0, t1 in trace.regions:
        hp.hpop_region_define(s, t0, t1)
    return s, keep


def engine_results(s, trace, flags=0):
    trees = hp.hpop_metrics_compute_all(s, flags)
    R = trace.n_hosts + trace.n_devices
    times = np.zeros((len(trace.regions), R, 4), np.int64)
    for g in range(len(trace.regions)):
        for r in range(R):
            times[g, r] = hp.hpop_resource_times(s, g, r)
    sums = np.array([hp.tree_sums(t) for t in trees], np.int64).reshape(len(trees), 10)
    ratios = np.array([hp.tree_ratios(t) for t in trees], np.float64).reshape(len(trees), 9)
    mask = np.array([t.undefined_mask for t in trees], np.uint32)
    return {"times": times, "sums": sums, "ratios": ratios, "mask": mask, "trees": trees}


def run_engine(trace, device=False, tuning=None, flags=0):
    s, keep = new_session(trace, device=device, tuning=tuning)
    try:
        return engine_results(s, trace, flags)
    finally:
        hp.hpop_session_destroy(s)


def assert_same(got, want, what=""):
    np.testing.assert_array_equal(got["times"], want["times"], err_msg="times " + what)
    np.testing.assert_array_equal(got["sums"], want["sums"], err_msg="sums " + what)
    # same exact integers, one IEEE division each: bit-identical ratios
    np.testing.assert_array_equal(got["ratios"].view(np.int64), want["ratios"].view(np.int64),
                                  err_msg="ratios " + what)
    np.testing.assert_array_equal(got["mask"], want["mask"], err_msg="mask " + what)
