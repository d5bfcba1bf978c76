"""Failure handling at the C ABI: every invalid input gets its status code
(GPU: validation runs on the device; every kernel stays in bounds)."""

import numpy as np
import pytest

from gpu_common import lib
from sfairsc_inputs import random_sparse_graph

pytestmark = pytest.mark.gpu


def _base():
    g = random_sparse_graph(200, 6, seed=1, h=3)
    return g.rowptr.copy(), g.col.copy(), g.val.copy(), g.groups.copy()


def _create(sf, rp, ci, va, gr, h=3, normalized=False):
    return sf.Graph(rp, ci, va, gr, h, normalized)


def test_valid_graph():
    sf = lib()
    _create(sf, *_base())


def test_asymmetric_value():
    sf = lib()
    rp, ci, va, gr = _base()
    va[5] += 0.25
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp, ci, va, gr)
    assert e.value.code == sf.E_ASYM


def _drop_entry(rp, ci, va, e):
    keep = np.ones(len(ci), bool)
    keep[e] = False
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))[keep]
    rp2 = np.zeros_like(rp)
    np.cumsum(np.bincount(rows, minlength=len(rp) - 1), out=rp2[1:])
    return rp2, ci[keep], va[keep]


@pytest.mark.parametrize("side", ["above", "below"])
def test_asymmetric_pattern_either_side(side):
    # one stored copy of an edge removed, above or below the diagonal: a
    # lookup from above finds no partner, or the counts above and below differ
    sf = lib()
    rp, ci, va, gr = _base()
    rows = np.repeat(np.arange(200), np.diff(rp))
    cand = np.flatnonzero(ci > rows) if side == "above" else np.flatnonzero(ci < rows)
    rp2, ci2, va2 = _drop_entry(rp, ci, va, cand[len(cand) // 2])
    for normalized in (False, True):
        with pytest.raises(sf.SfairscError) as e:
            _create(sf, rp2, ci2, va2, gr, normalized=normalized)
        assert e.value.code == sf.E_ASYM


@pytest.mark.parametrize("side", ["above", "below"])
def test_asymmetric_value_either_side(side):
    sf = lib()
    rp, ci, va, gr = _base()
    rows = np.repeat(np.arange(200), np.diff(rp))
    cand = np.flatnonzero(ci > rows) if side == "above" else np.flatnonzero(ci < rows)
    va[cand[-1]] = np.nextafter(va[cand[-1]], va.dtype.type(np.inf))  # one ulp of the stored dtype
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp, ci, va, gr)
    assert e.value.code == sf.E_ASYM


def test_negative_and_nan_weights():
    sf = lib()
    for bad in (-1.0, np.nan, np.inf):
        rp, ci, va, gr = _base()
        va[3] = bad
        with pytest.raises(sf.SfairscError) as e:
            _create(sf, rp, ci, va, gr)
        assert e.value.code == sf.E_ARG


def test_empty_group_and_bad_label():
    sf = lib()
    rp, ci, va, gr = _base()
    gr[gr == 2] = 1
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp, ci, va, gr)
    assert e.value.code == sf.E_EMPTY_GROUP
    rp, ci, va, gr = _base()
    gr[0] = 7
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp, ci, va, gr)
    assert e.value.code == sf.E_ARG


def test_isolated_vertex_normalized_only():
    sf = lib()
    rp, ci, va, gr = _base()
    # drop every edge of vertex 0 (and the mirrored copies)
    rows = np.repeat(np.arange(200), np.diff(rp))
    keep = (rows != 0) & (ci != 0)
    rows, ci2, va2 = rows[keep], ci[keep], va[keep]
    rp2 = np.zeros(201, np.int32)
    np.cumsum(np.bincount(rows, minlength=200), out=rp2[1:])
    _create(sf, rp2, ci2, va2, gr, normalized=False)
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp2, ci2, va2, gr, normalized=True)
    assert e.value.code == sf.E_ISOLATED


def test_malformed_csr():
    sf = lib()
    rp, ci, va, gr = _base()
    rp2 = rp.copy()
    rp2[10], rp2[11] = rp2[11], rp2[10]  # decreasing row pointers
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp2, ci, va, gr)
    assert e.value.code == sf.E_ARG
    ci2 = ci.copy()
    a, b = rp[4], rp[5]
    ci2[a:b] = ci2[a:b][::-1]  # unsorted row
    if b - a >= 2:
        with pytest.raises(sf.SfairscError) as e:
            _create(sf, rp, ci2, va, gr)
        assert e.value.code == sf.E_ARG
    ci3 = ci.copy()
    ci3[rp[7]] = 7  # diagonal entry
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp, ci3, va, gr)
    assert e.value.code in (sf.E_ARG, sf.E_ASYM)


STRUCTURE_CASES = {
    # name: how the CSR of the valid 200-vertex graph is broken
    "rowptr_first": lambda rp, ci: rp.__setitem__(0, 1),
    "rowptr_last_short": lambda rp, ci: rp.__setitem__(-1, rp[-1] - 1),
    "rowptr_beyond_nnz": lambda rp, ci: rp.__setitem__(50, rp[-1] + 1000),
    "rowptr_negative": lambda rp, ci: rp.__setitem__(30, -5),
    "rowptr_int_min": lambda rp, ci: rp.__setitem__(30, np.iinfo(np.int32).min),
    "col_equal_n": lambda rp, ci: ci.__setitem__(7, 200),
    "col_negative": lambda rp, ci: ci.__setitem__(7, -1),
    "col_int_max": lambda rp, ci: ci.__setitem__(7, np.iinfo(np.int32).max),
}


@pytest.mark.parametrize("name", sorted(STRUCTURE_CASES))
@pytest.mark.parametrize("normalized", [False, True])
def test_malformed_structure_is_rejected(name, normalized):
    # the set-up passes run without a host check between them, so each of
    # these reaches every pass, whose own guards keep it in bounds
    sf = lib()
    rp, ci, va, gr = _base()
    STRUCTURE_CASES[name](rp, ci)
    with pytest.raises(sf.SfairscError) as e:
        _create(sf, rp, ci, va, gr, normalized=normalized)
    assert e.value.code == sf.E_ARG, name
    # the library is still usable afterwards
    _create(sf, *_base(), normalized=normalized).close()


def test_bad_solver_arguments():
    sf = lib()
    G = _create(sf, *_base())
    with pytest.raises(sf.SfairscError) as e:
        G.eigs(0)
    assert e.value.code == sf.E_ARG
    with pytest.raises(sf.SfairscError) as e:
        G.eigs(199)
    assert e.value.code == sf.E_ARG
    with pytest.raises(sf.SfairscError) as e:
        G.eigs(4, block_width=5)
    assert e.value.code == sf.E_ARG


# --- the library rejects exactly the inputs the oracle's validation rejects ---


def _scipy(rp, ci, va, n=200):
    import scipy.sparse as sp

    return sp.csr_matrix((np.asarray(va, np.float64), ci, rp), shape=(n, n))


def _case(name):
    rp, ci, va, gr = _base()
    normalized = False
    if name == "asym_value":
        va[5] += 0.25
    elif name == "asym_pattern":
        # drop the mirror of one stored entry: (i, j) kept, (j, i) removed
        i = 3
        j = int(ci[rp[i]])
        rows = np.repeat(np.arange(200), np.diff(rp))
        pos = np.nonzero((rows == j) & (ci == i))[0][0]
        keep = np.ones(ci.size, bool)
        keep[pos] = False
        ci, va, rows = ci[keep], va[keep], rows[keep]
        rp = np.zeros(201, np.int32)
        np.cumsum(np.bincount(rows, minlength=200), out=rp[1:])
    elif name in ("negative", "nan", "inf"):
        bad = {"negative": -1.0, "nan": np.nan, "inf": np.inf}[name]
        i = 3
        j = int(ci[rp[i]])
        rows = np.repeat(np.arange(200), np.diff(rp))
        va[rp[i]] = bad
        va[np.nonzero((rows == j) & (ci == i))[0][0]] = bad  # both copies: symmetric
    elif name == "diagonal":
        # insert a stored w_77 = 1
        rows = np.repeat(np.arange(200), np.diff(rp))
        rows = np.append(rows, 7)
        ci = np.append(ci, 7).astype(np.int32)
        va = np.append(va, 1.0)
        o = np.lexsort((ci, rows))
        rows, ci, va = rows[o], ci[o], va[o]
        rp = np.zeros(201, np.int32)
        np.cumsum(np.bincount(rows, minlength=200), out=rp[1:])
    elif name == "label":
        gr[0] = 7
    elif name == "empty_group":
        gr[gr == 2] = 1
    elif name == "isolated_normalized":
        rows = np.repeat(np.arange(200), np.diff(rp))
        keep = (rows != 0) & (ci != 0)
        rows, ci, va = rows[keep], ci[keep], va[keep]
        rp = np.zeros(201, np.int32)
        np.cumsum(np.bincount(rows, minlength=200), out=rp[1:])
        normalized = True
    return rp, ci.astype(np.int32), va, gr, normalized


@pytest.mark.parametrize("name", ["valid", "asym_value", "asym_pattern", "negative", "nan", "inf", "diagonal",
                                  "label", "empty_group", "isolated_normalized"])
def test_rejects_what_the_oracle_rejects(name):
    import oracle

    sf = lib()
    rp, ci, va, gr, normalized = _case(name)
    try:
        oracle.validate_graph(_scipy(rp, ci, va), gr, 3, normalized=normalized)
        oracle_ok = True
    except ValueError:
        oracle_ok = False
    try:
        G = _create(sf, rp, ci, va, gr, normalized=normalized)
        G.close()
        lib_ok = True
    except sf.SfairscError:
        lib_ok = False
    assert oracle_ok == lib_ok == (name == "valid"), (name, oracle_ok, lib_ok)


def test_k_bound_matches_the_oracle():
    import oracle

    sf = lib()
    rp, ci, va, gr = _base()
    W = _scipy(rp, ci, va)
    G = _create(sf, rp, ci, va, gr)
    for k in (0, 200 - 3 + 2):
        with pytest.raises(ValueError, match="k out of range"):
            oracle.validate_graph(W, gr, 3, k=k)
        with pytest.raises(sf.SfairscError) as e:
            G.eigs(k)
        assert e.value.code == sf.E_ARG
