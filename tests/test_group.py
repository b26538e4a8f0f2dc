"""Group plans (several patterns as one block-diagonal matrix): the symbolic
result of every block equals the oracle's analysis of that pattern alone,
shifted to the block's offset; block offsets, sizes and argument checks."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.test_abi import check_supernode_invariants


def _members():
    return [W.small_grid((6, 6), "nd", seed=71),
            W.small_grid((9, 7), "natural", seed=72),
            W.small_grid((4, 4, 4), "nd", seed=73),
            W.random_spd(57, 0.06, seed=74),
            W.small_grid((5, 5, 3), "nd", seed=75)]


def _group(ws, **opts):
    import paper_2110_12865_amd as S
    return S.analyze_group([(w.pattern.colptr, w.pattern.rowind, w.perm) for w in ws], **opts)


class _Concat:
    """The oracle's symbolic result of the block-diagonal matrix, assembled
    from the per-pattern results (a block-diagonal matrix has a forest of
    independent elimination trees)."""

    def __init__(self, syms, col0):
        self.n = int(col0[-1])
        self.parent = np.concatenate([np.where(s.parent >= 0, s.parent + c, -1)
                                      for s, c in zip(syms, col0[:-1])]).astype(np.int32)
        cnt = np.concatenate([np.diff(s.Lcolptr) for s in syms])
        self.Lcolptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        self.Lrowind = np.concatenate([s.Lrowind + c for s, c in zip(syms, col0[:-1])])


@pytest.mark.parametrize("relax", [1, 0])
def test_group_symbolic_equals_per_pattern_oracle(relax):
    ws = _members()
    plan = _group(ws, relax=relax)
    col0, val0 = plan.export_blocks()
    assert np.array_equal(col0, np.concatenate([[0], np.cumsum([w.pattern.n for w in ws])]))
    assert np.array_equal(val0, np.concatenate([[0], np.cumsum([w.pattern.nnz for w in ws])]))
    syms = [oracle.symbolic(w.pattern.n, w.pattern.colptr, w.pattern.rowind, w.perm) for w in ws]
    perm, parent, Lcolptr, Lrowind = plan.export_symbolic()
    for k, (w, s) in enumerate(zip(ws, syms)):
        c0, c1 = col0[k], col0[k + 1]
        ref = np.arange(w.pattern.n) if w.perm is None else w.perm
        assert np.array_equal(perm[c0:c1], ref + c0)
        assert np.array_equal(parent[c0:c1], np.where(s.parent >= 0, s.parent + c0, -1))
        assert np.array_equal(np.diff(Lcolptr[c0:c1 + 1]), np.diff(s.Lcolptr))
        assert np.array_equal(Lrowind[Lcolptr[c0]:Lcolptr[c1]], s.Lrowind + c0)
    inf = plan.info()
    assert inf["nblocks"] == len(ws)
    assert inf["nnzL"] == sum(s.nnzL for s in syms)
    assert inf["flops"] == pytest.approx(sum(s.flops() for s in syms), rel=1e-12)
    check_supernode_invariants(plan, _Concat(syms, col0))
    # no supernode spans two blocks
    first = plan.export_supernodes()[0]
    blk = np.searchsorted(col0, first[:-1], side="right") - 1
    blk_last = np.searchsorted(col0, first[1:] - 1, side="right") - 1
    assert np.array_equal(blk, blk_last)


def test_single_pattern_group_equals_plain_plan():
    import paper_2110_12865_amd as S
    w = W.small_grid((8, 8, 8), "nd", seed=76)
    p = w.pattern
    a = S.analyze(p.colptr, p.rowind, w.perm)
    g = _group([w])
    for x, y in zip(a.export_symbolic(), g.export_symbolic()):
        assert np.array_equal(x, y)
    for x, y in zip(a.export_supernodes(), g.export_supernodes()):
        assert np.array_equal(x, y)
    assert a.info() == g.info()


def test_uneven_batch_configuration_sizes():
    """The eight patterns of the uneven-batch configuration as one group:
    sizes add up to the per-pattern oracle's."""
    ws = W.config(3, batch=1)
    plan = _group(ws)
    inf = plan.info()
    syms = [oracle.symbolic(w.pattern.n, w.pattern.colptr, w.pattern.rowind, w.perm) for w in ws]
    assert inf["n"] == sum(w.pattern.n for w in ws) == 41920
    assert inf["nnzA"] == sum(w.pattern.nnz for w in ws)
    assert inf["nnzL"] == sum(s.nnzL for s in syms)
    assert inf["nblocks"] == 8
    # the deepest pattern sets the number of levels
    depth = [_group([w]).info()["nlevels"] for w in ws]
    assert inf["nlevels"] == max(depth)


def test_group_argument_checks():
    import paper_2110_12865_amd as S
    ws = _members()[:2]
    p0, p1 = ws[0].pattern, ws[1].pattern
    with pytest.raises(ValueError):
        S.analyze_group([])
    # a row index of pattern 1 beyond its own order (still inside the group)
    bad = p1.rowind.copy()
    bad[-1] = p1.n
    with pytest.raises(S.SpcholError) as e:
        S.analyze_group([(p0.colptr, p0.rowind), (p1.colptr, bad)])
    assert e.value.status == S.SC_EPATTERN
    # a permutation entry outside its own pattern
    perm = np.arange(p0.n, dtype=np.int32)
    perm[0] = p0.n
    with pytest.raises(S.SpcholError) as e:
        S.analyze_group([(p0.colptr, p0.rowind, perm), (p1.colptr, p1.rowind)])
    assert e.value.status == S.SC_EPATTERN
    # a repeated permutation entry
    perm = np.arange(p0.n, dtype=np.int32)
    perm[1] = 0
    with pytest.raises(S.SpcholError) as e:
        S.analyze_group([(p0.colptr, p0.rowind, perm), (p1.colptr, p1.rowind)])
    assert e.value.status == S.SC_EPATTERN
    # missing diagonal in one member
    with pytest.raises(S.SpcholError) as e:
        S.analyze_group([(p0.colptr, p0.rowind), (p1.colptr, p1.rowind[::-1].copy())])
    assert e.value.status == S.SC_EPATTERN
