"""Device projection A^dag H A (Sec. II A, Fig. 2) against the oracle's convention route,
entry by entry, and the S_n closed form."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import basis as obasis
from tests._common import oracle_blocks

pytestmark = pytest.mark.gpu


def _terms(n):
    h0 = W.heisenberg_ring_terms(0.83, 0.37) + [W.ring_pair(0.21, "zz", min(2, n // 2) or 1)]
    hk = [[W.one_body(1.0, "x")], [W.one_body(1.0, "y")], [W.ring_pair(0.5, "xx")]]
    return h0, hk


@pytest.mark.parametrize("n,stride,group", [(3, 1, "dihedral"), (4, 1, "dihedral"), (5, 1, "dihedral"),
                                            (6, 1, "dihedral"), (8, 1, "dihedral"), (6, 1, "cyclic"),
                                            (7, 1, "cyclic"), (10, 1, "dihedral")])
def test_blocks_entrywise(lib, n, stride, group):
    print(f"project n={n} stride={stride} {group}", flush=True)
    h0, hk = _terms(n)
    B = lib.Basis(n, group, stride)
    S = lib.System(B, h0, hk)
    ob = oracle_blocks(n, h0, hk, group, stride)
    assert [b["m"] for b in ob] == B.sizes
    for b, blk in enumerate(ob):
        for op in range(len(hk) + 1):
            got = S.block(b, op).cpu().numpy()
            want = blk["H0"] if op == 0 else blk["Hk"][op - 1]
            assert np.abs(got - want).max() < 1e-12, (blk["label"], op)


def test_staggered_controls_two_site_group(lib):
    n = 8
    hk = [[W.one_body(1.0, "z", stagger=True)], [W.one_body(1.0, "x", sites="even")]]
    h0 = W.heisenberg_ring_terms(1.0)
    B = lib.Basis(n, "dihedral", 2)
    S = lib.System(B, h0, hk)
    ob = oracle_blocks(n, h0, hk, "dihedral", 2)
    for b, blk in enumerate(ob):
        for op in range(3):
            want = blk["H0"] if op == 0 else blk["Hk"][op - 1]
            assert np.abs(S.block(b, op).cpu().numpy() - want).max() < 1e-12
    with pytest.raises(lib.QocError) as e:
        lib.System(lib.Basis(n, "dihedral", 1), h0, hk)
    assert e.value.status == 2


@pytest.mark.parametrize("n", [4, 7, 128])
def test_symmetric_blocks(lib, n):
    h0 = [W.one_body(0.9, "z"), W.all_pairs(0.3, "xx"), W.all_pairs(-0.2, "yy")]
    hk = [[W.one_body(1.0, "x")], [W.one_body(1.0, "y")]]
    B = lib.Basis(n, "symmetric")
    S = lib.System(B, h0, hk)
    ob = obasis.sn_blocks(n, h0)
    okx = obasis.sn_blocks(n, hk[0])
    for b in range(min(len(ob), 6)):
        assert np.abs(S.block(b, 0).cpu().numpy() - ob[b][1]).max() < 1e-9 * max(1.0, np.abs(ob[b][1]).max())
        assert np.abs(S.block(b, 1).cpu().numpy() - okx[b][1]).max() < 1e-12
