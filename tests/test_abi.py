"""The C-ABI library loads and exports every entry point its header declares
(host-only checks: no device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mdp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2109_00857_amd import mdp

    if not os.path.exists(mdp.LIB_PATH):
        from paper_2109_00857_amd import _build

        _build.build()
    return mdp.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 9, names
    for n in names:
        assert hasattr(lib, n), n
    from paper_2109_00857_amd import mdp

    assert sorted(mdp.EXPORTED) == names


def test_status_strings(lib):
    from paper_2109_00857_amd import mdp

    for s in range(7):
        assert mdp.mdp_status_str(s) != "unknown status"
    assert mdp.mdp_status_str(99) == "unknown status"


def test_query_sizes(lib):
    from paper_2109_00857_amd import mdp, workloads as W

    w = W.config2(nx=20, ny=10, nt=5, n_real=300, K=4, n_head=16)
    q = mdp.mdp_build_query(w.problem)
    assert q["n_states"] == 5 * 200
    assert q["n_actions"] == 16
    assert q["n_rows"] == 5 * 200 * 16
    assert q["n_sg"] == 25
    assert q["nnz_upper"] == q["n_rows"] * 25
    assert q["n_missions"] == 3
    assert q["scratch_bytes"] > q["n_states"] * 8


@pytest.mark.parametrize("field,value", [("nx", 0), ("n_modes", 17), ("n_real", 70000), ("n_head", 65),
                                         ("target_i", 99), ("dt", 0.0), ("mission_mask", 0),
                                         ("sub_hx", -1)])
def test_query_rejects_invalid(lib, field, value):
    from paper_2109_00857_amd import mdp, workloads as W

    w = W.config1(nt=2, n_real=10, sub_h=2)
    p = dict(w.problem)
    p[field] = value
    with pytest.raises(mdp.MdpError):
        mdp.mdp_build_query(p)


def test_query_rejects_oversized_subgrid(lib):
    from paper_2109_00857_amd import mdp, workloads as W

    w = W.config1(nt=2, n_real=10, sub_h=40)
    with pytest.raises(mdp.MdpError):
        mdp.mdp_build_query(w.problem)


def test_autotune_query_sizes(lib):
    """The tuning sample's scratch is sized on the host; invalid problems are refused."""
    import ctypes as C

    from paper_2109_00857_amd import mdp, workloads as W

    w = W.config2()
    n = C.c_size_t()
    assert lib.mdp_autotune_query(C.byref(mdp.problem_struct(w.problem)), C.byref(n)) == mdp.MDP_OK
    sz = mdp.mdp_build_query(w.problem)
    assert 0 < n.value < sz["n_rows"] * 40 + sz["scratch_bytes"]
    bad = dict(w.problem, nx=0)
    assert lib.mdp_autotune_query(C.byref(mdp.problem_struct(bad)), C.byref(n)) == mdp.MDP_E_INVALID
