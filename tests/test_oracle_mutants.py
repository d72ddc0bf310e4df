"""Planted mistakes in the oracle (rebuilt on the CPU from a modified copy of
its source) must each fail at least one pin: the brute-force reading, the
PILS tables or a closed form. This shows the pins can see a dropped term, a
wrong sign or index, or a transposed operand anywhere in the oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import tracegen as tg
import pils
from brute import occupancy_times, tree_from_times

SRC = os.path.join(os.path.dirname(oracle.__file__), "hpop_oracle.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("merge drops the running max", "cur.e = orc_max(cur.e, v[i].e);", "cur.e = v[i].e;"),
    ("no clip at region start", "int64_t a = orc_max(v[j].s, t0[r]);", "int64_t a = v[j].s;"),
    ("no clip at region end", "int64_t b = orc_min(v[j].e, t1[r]);", "int64_t b = v[j].e;"),
    ("offloading not differenced", "out[1] = d2 - d1;\n                out[2] = d3 - d2;",
     "out[1] = d2;\n                out[2] = d3 - d2;"),
    ("idle from the wrong level", "out[2] = E - d2;", "out[2] = E - d1;"),
    ("other from the wrong level", "out[3] = E - d3;", "out[3] = E - d2;"),
    ("MPI LB numerator", "q[2] = orc_ratio(sUW, n * mUW", "q[2] = orc_ratio(sU, n * mUW"),
    ("device CE transposed", "q[7] = orc_ratio(mK, mKM", "q[7] = orc_ratio(mKM, mK"),
    ("device LB uses n", "q[6] = orc_ratio(sK, m * mK", "q[6] = orc_ratio(sK, n * mK"),
    ("MPI ranked as offloading", "case ORC_HOST_MPI: return 2;", "case ORC_HOST_MPI: return 1;"),
    ("memop ranked as kernel", "case ORC_DEV_MEMOP: return 1;", "case ORC_DEV_MEMOP: return 0;"),
    ("level test inverted", "if (orc_rank(J->g_kind[i]) <= L", "if (orc_rank(J->g_kind[i]) == L"),
    ("0/0 taken as 0", "        return 1.0;\n    }\n    return (double)num", "        return 0.0;\n    }\n    return (double)num"),
    ("max K+M drops M", "mKM = orc_max(mKM, x[0] + x[1]);", "mKM = orc_max(mKM, x[0]);"),
    ("sum U+W drops W", "sUW += x[0] + x[1];", "sUW += x[0];"),
    ("host PE over m", "q[0] = orc_ratio(sU, n * E", "q[0] = orc_ratio(sU, m * E"),
    ("orchestration uses max K", "q[8] = orc_ratio(mKM, E", "q[8] = orc_ratio(mK, E"),
]


def _pins_fail(lib):
    """True if some pin rejects the oracle loaded from `lib`."""
    try:
        for seed in range(60):
            rng = np.random.default_rng(seed)
            tr = tg.random_tiny(rng, max_span=int(rng.integers(2, 60)), max_events=int(rng.integers(1, 12)))
            got = oracle.compute(tr, lib=lib)
            want = occupancy_times(tr)
            if not np.array_equal(got["times"], want):
                return True
            sums, ratios, mask = tree_from_times(want, tr.n_hosts, tr.n_devices, tr.regions)
            if not (np.array_equal(got["sums"], sums) and np.array_equal(got["ratios"], ratios)
                    and np.array_equal(got["mask"], mask)):
                return True
        for name, printed, t in pils.load():
            q = oracle.compute(pils.build_trace(t), lib=lib)["ratios"][0]
            if np.any(np.abs(q - np.array(printed)) > 0.005 + 1e-12):
                return True
    except oracle.OracleError:
        return True
    return False


def test_unmodified_oracle_passes_the_pins():
    assert not _pins_fail(None)


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda m: m[0])
def test_planted_mistake_is_caught(mutant, tmp_path):
    name, old, new = mutant
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-I", os.path.dirname(SRC), "-o", str(so), str(path),
                           "-lpthread"])
    lib = oracle.load_library(str(so))
    assert _pins_fail(lib), "planted mistake not caught: " + name
