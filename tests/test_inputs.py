"""Input generator checks: the twisted-bilayer geometry against the paper's
Table 2 and atom counts, and the structural promises of the pattern and D."""
import math
import os

import numpy as np
import pytest

from paper_2409_09399_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table2_lattice_vectors.txt")


def _table2():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [float(x) for x in line.split()]
        rows.append((int(v[0]), np.array(v[1:4]), np.array(v[4:7]), np.array(v[7:10])))
    return rows


@pytest.mark.parametrize("row", _table2(), ids=lambda r: str(r[0]))
def test_tbg_matches_table2(row):
    """Atom count and in-plane cell of the commensurate bilayer reproduce the
    paper's Table 2 (a = 2.4595 Angstrom gives the printed lengths)."""
    n, X, Y, Z = row
    q = n // 4
    i = int(round((-3 + math.sqrt(9 - 12 * (1 - q))) / 6))
    assert I.tbg_atom_count(i) == n
    cell, pos, theta = I.tbg(i, a_ang=2.4595)
    assert pos.shape[0] == n
    L = np.linalg.norm(cell[0]) / I.BOHR_PER_ANGSTROM
    assert abs(L - np.linalg.norm(X)) < 2e-3
    assert abs(L - np.linalg.norm(Z)) < 2e-3
    # the printed in-plane vectors are 60 degrees apart, Y is orthogonal to both
    assert abs(X @ Z / (np.linalg.norm(X) * np.linalg.norm(Z)) - 0.5) < 1e-3
    assert abs(X @ Y) < 1e-2 * np.linalg.norm(X) * np.linalg.norm(Y)
    assert abs(np.linalg.norm(Y) - 30.0) < 1e-2
    c = cell[0] @ cell[1] / (np.linalg.norm(cell[0]) * np.linalg.norm(cell[1]))
    assert abs(c - 0.5) < 1e-12


def test_tbg_no_duplicate_atoms_and_bond_length():
    cell, pos, theta = I.tbg(2, a_ang=2.46)
    # minimum in-layer distance is the C-C bond a/sqrt(3)
    layer0 = pos[pos[:, 2] < 1.0]
    best = np.inf
    for T in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [0], indexing="ij")).reshape(3, -1).T:
        d = layer0[:, None, :] - (layer0[None, :, :] + T @ cell)
        r = np.linalg.norm(d, axis=2)
        if not T.any():
            r[np.arange(r.shape[0]), np.arange(r.shape[0])] = np.inf
        best = min(best, r.min())
    assert abs(best - 2.46 * I.BOHR_PER_ANGSTROM / math.sqrt(3)) < 1e-9
    assert abs(math.degrees(theta) - 13.1736) < 1e-3


def test_pattern_transpose_closed_and_d_symmetric():
    s = I.diamond8(0, grid=(8, 8, 8))
    idx = I.block_index(s.blk_i, s.blk_j, s.blk_r)
    norb = s.norb_atom()
    for k in range(len(s.blk_i)):
        i, j, r = int(s.blk_i[k]), int(s.blk_j[k]), s.blk_r[k]
        kt = idx[(j, i, -int(r[0]), -int(r[1]), -int(r[2]))]
        ni, nj = int(norb[i]), int(norb[j])
        a = s.d[s.blk_off[k]:s.blk_off[k] + ni * nj].reshape(ni, nj)
        b = s.d[s.blk_off[kt]:s.blk_off[kt] + ni * nj].reshape(nj, ni)
        assert np.array_equal(a, b.T)
    # every pair closer than the sum of cutoffs is present
    rc = s.rcut_atom()
    for i in range(s.natom):
        for j in range(s.natom):
            for r in np.array(np.meshgrid(*[np.arange(-3, 4)] * 3, indexing="ij")).reshape(3, -1).T:
                d = np.linalg.norm(s.pos[j] + r @ s.cell - s.pos[i])
                if d < rc[i] + rc[j]:
                    assert (i, j, int(r[0]), int(r[1]), int(r[2])) in idx


def test_generator_is_deterministic():
    a = I.diamond8(3, grid=(8, 8, 8))
    b = I.diamond8(3, grid=(8, 8, 8))
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.d, b.d) and np.array_equal(a.v, b.v)
    assert np.array_equal(a.species_list[0].f, b.species_list[0].f)
