"""The C ABI library loads, exports every symbol include/gint.h declares, and
rejects invalid inputs with the documented codes before touching the GPU
(no compute calls here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def _declared():
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if f.endswith(".h"):
            txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(gint_[a-z_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def G():
    from paper_2409_09399_amd import gint
    return gint


def test_exports_every_declared_symbol(G):
    lib = C.CDLL(G.LIB_PATH)
    names = _declared()
    assert "gint_vlocal" in names and "gint_rho" in names and "gint_force_stress" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(G.EXPORTED) == set(names)


def test_strerror(G):
    for code in (0, -1, -2, -3, -4, -5):
        assert len(G._lib.gint_strerror(code)) > 0


def _tiny():
    from paper_2409_09399_amd import inputs as I
    return I.diamond8(0, grid=(8, 8, 8))


def _create(G, s, **kw):
    try:
        G.Plan(s, **kw)
    except G.GintError as e:
        return e.code
    return 0


def test_rejects_bad_inputs(G):
    s = _tiny()
    t = _tiny(); t.pos = t.pos.copy(); t.pos[3, 1] = np.nan
    assert _create(G, t) == G.GINT_EINVAL
    t = _tiny(); t.grid = np.array([8, 0, 8], np.int32)
    assert _create(G, t) == G.GINT_EINVAL
    t = _tiny(); t.species = t.species.copy(); t.species[0] = 5
    assert _create(G, t) == G.GINT_EINVAL
    t = _tiny(); t.cell = np.zeros((3, 3))
    assert _create(G, t) == G.GINT_EINVAL
    assert _create(G, s, cluster_atoms=9) == G.GINT_EINVAL
    # clusters of more than four atoms: only mixed-precision plans with rho and force on bricks
    assert _create(G, s, cluster_atoms=5) == G.GINT_EINVAL
    assert _create(G, s, cluster_atoms=8, precision=G.GINT_MIXED_FP16X3, decomposition=1) == G.GINT_EINVAL
    assert _create(G, s, precision=7) == G.GINT_EUNSUPPORTED


def test_rejects_unsupported_basis(G):
    from paper_2409_09399_amd import inputs as I
    rng = np.random.default_rng(0)
    t = _tiny()
    t.species_list = [I.make_species("F", (0, 3), 6.0, 0.01, rng)]
    assert _create(G, t) == G.GINT_EUNSUPPORTED
    t.species_list = [I.make_species("G", (0, 0, 1, 1, 2, 2), 6.0, 0.01, rng)]   # 18 orbitals
    assert _create(G, t) == G.GINT_EUNSUPPORTED


def test_rejects_pattern_not_transpose_closed(G):
    s = _tiny()
    keep = np.ones(len(s.blk_i), bool)
    # drop one off-diagonal block but keep its transpose
    k = int(np.nonzero(s.blk_i != s.blk_j)[0][0])
    keep[k] = False
    s.blk_i, s.blk_j, s.blk_r, s.blk_off = s.blk_i[keep], s.blk_j[keep], s.blk_r[keep], s.blk_off[keep]
    assert _create(G, s) == G.GINT_EPATTERN


def test_rejects_missing_overlapping_pair(G):
    from paper_2409_09399_amd import inputs as I
    s = _tiny()
    # remove a close pair (both directions): orbitals overlap on grid points
    d = np.linalg.norm(s.pos[s.blk_j] + s.blk_r @ s.cell - s.pos[s.blk_i], axis=1)
    k = int(np.nonzero((s.blk_i != s.blk_j) & (d < 4.0))[0][0])
    i, j, r = s.blk_i[k], s.blk_j[k], s.blk_r[k]
    drop = ((s.blk_i == i) & (s.blk_j == j) & np.all(s.blk_r == r, axis=1)) | \
           ((s.blk_i == j) & (s.blk_j == i) & np.all(s.blk_r == -r, axis=1))
    keep = ~drop
    s.blk_i, s.blk_j, s.blk_r = s.blk_i[keep], s.blk_j[keep], s.blk_r[keep]
    s.blk_off = I.block_offsets(s.blk_i, s.blk_j, s.norb_atom())
    assert _create(G, s) == G.GINT_EPATTERN


def test_rejects_duplicate_and_overlapping_blocks(G):
    s = _tiny()
    t = _tiny()
    t.blk_i = np.concatenate([s.blk_i, s.blk_i[:1]]); t.blk_j = np.concatenate([s.blk_j, s.blk_j[:1]])
    t.blk_r = np.concatenate([s.blk_r, s.blk_r[:1]]); t.blk_off = np.concatenate([s.blk_off, [s.nnz]])
    assert _create(G, t) == G.GINT_EINVAL
    t = _tiny(); t.blk_off = t.blk_off.copy(); t.blk_off[1] = t.blk_off[0] + 1
    assert _create(G, t) == G.GINT_EINVAL


def test_batch_errors_name_the_system(G):
    """A batch fails as a whole when any system is invalid; nothing is built."""
    good = _tiny()
    bad = _tiny(); bad.grid = np.array([8, 8, -1], np.int32)
    assert _create(G, [good, bad]) == G.GINT_EINVAL
    bad = _tiny()
    keep = np.ones(len(bad.blk_i), bool); keep[5] = False
    bad.blk_i, bad.blk_j, bad.blk_r = bad.blk_i[keep], bad.blk_j[keep], bad.blk_r[keep]
    bad.blk_off = bad.blk_off[keep]
    assert _create(G, [good, bad, good]) == G.GINT_EPATTERN
    with pytest.raises(ValueError):
        G.Plan([])


def test_null_arguments(G):
    lib = G._lib
    sts, keep, n = G._marshal_batch(_tiny())
    opt = G.gint_options()
    out = C.c_void_p()
    assert lib.gint_plan_create(C.byref(out), sts, 0, C.byref(opt), None) == G.GINT_EINVAL
    assert lib.gint_plan_create(None, sts, 1, C.byref(opt), None) == G.GINT_EINVAL
    assert lib.gint_graph_create(C.byref(out), None, *([None] * 8)) == G.GINT_EINVAL
    assert lib.gint_graph_launch(None, None) == G.GINT_EINVAL
    rep = G.gint_tune_report()
    assert lib.gint_autotune(sts, 1, None, 1.0, None, C.byref(rep)) == G.GINT_EINVAL
    assert lib.gint_autotune(sts, 1, C.byref(opt), -1.0, None, C.byref(rep)) == G.GINT_EINVAL
    assert lib.gint_plan_query_system(None, 0, C.byref(G.gint_system_sizes())) == G.GINT_EINVAL
    lib.gint_graph_destroy(None)
    lib.gint_plan_destroy(None)


def test_device_cap_gives_enomem_before_any_hip_call(G):
    """A plan larger than the caller's device-memory cap fails with
    GINT_ENOMEM; the check runs on the host plan before the device is
    touched (so it holds here, without a GPU)."""
    from paper_2409_09399_amd import inputs as I
    s = I.diamond8(0)            # grid 32^3: a plan of a few MiB
    assert _create(G, s, device_mib_cap=1) == G.GINT_ENOMEM
    # the cap applies to a batch as a whole
    t = _tiny()
    assert _create(G, [t, s, t], device_mib_cap=1) == G.GINT_ENOMEM
