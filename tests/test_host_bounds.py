"""The interval analysis behind the lazy reduction (csrc/bounds.py) runs, and
its constants are the ones the kernels use.

bounds.py replays every XYZZ formula on upper bounds of values and limbs; it is
only a proof of the kernels if the subtraction multiples it assumes are the
ones curve.h passes to sub_k, in the same order, and if its borrowed-limb
tables equal the K constants of field_constants.h.  Both are read from the
sources here, so a change to either side without the other fails.
"""
import importlib.util
import os
import re

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2507_07031_amd", "csrc")


@pytest.fixture(scope="module")
def bounds():
    spec = importlib.util.spec_from_file_location("zk_bounds", os.path.join(CSRC, "bounds.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _read(name):
    with open(os.path.join(CSRC, name)) as fh:
        return fh.read()


def _function_body(src, signature):
    i = src.index(signature)
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        depth += {"{": 1, "}": -1}.get(src[k], 0)
        if depth == 0:
            return src[j:k + 1]
    raise AssertionError("unterminated body of " + signature)


def test_interval_analysis_holds(bounds):
    out = bounds.check_all()
    assert set(out) == {"madd", "add", "dbl"}


def test_sub_multiples_match_curve_formulas(bounds):
    src = _read("curve.h")
    # the subtraction multiples of each formula, in source order (an inner
    # sub_k's multiple is written before the outer one's), against the names
    # bounds.py gives them in the order its replay performs them
    order = {
        "ZK_HD xyzz madd(": ["madd.P", "madd.R", "madd.X3", "madd.QX", "madd.nY1"],
        "ZK_HD xyzz madd_signed(": ["madd.P", "madd.R", "madd.X3", "madd.QX", "madd.nY1"],
        "ZK_HD xyzz add(const xyzz& a, const xyzz& b)": ["add.P", "add.R", "add.X3", "add.QX", "add.nS1"],
        "ZK_HD xyzz dbl(": ["dbl.X3", "dbl.SX", "dbl.Y3"],
    }
    for sig, names in order.items():
        body = _function_body(src, sig)
        used = re.findall(r"Fq::([KH]\d+)", body)
        assert used == [bounds.SUB_K[n] for n in names], (sig, used)


def test_borrowed_tables_match_field_constants(bounds):
    src = _read("field_constants.h")
    fq = src[src.index("struct FqP"):src.index("struct FrP")]
    for name, c, fn in [("K%d" % c, c, bounds.borrowed) for c in (1, 2, 4, 8, 16)] + [("H8", 8, bounds.borrowed30)]:
        m = re.search(r"%s\[9\] = \{([^}]*)\}" % name, fq)
        assert m, name
        words = [int(w.strip().rstrip("u"), 16) for w in m.group(1).split(",")]
        assert words == fn(c * bounds.P), name
