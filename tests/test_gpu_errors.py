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
