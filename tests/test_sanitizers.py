"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only).  Two standalone programs (tests/native) are built with gcc/g++ and
-fsanitize=address,undefined: one runs the FP64 oracle on a dumped system
(its outputs must equal those of the oracle library the other tests use),
the other runs the plan builder (gint_plan.cpp, compiled without HIP) and
checks its bigcell-stationary bricks against brute force.  Any sanitizer
report fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="needs gcc/g++")


def dump(system, d):
    """The arrays of a System in the drivers' raw format."""
    s = system
    sps = s.species_list
    nch = [sp.nchan for sp in sps]
    chan_off = np.concatenate([[0], np.cumsum(nch)]).astype(np.int32)
    tabs_f, tabs_fp, tab_off, o = [], [], [], 0
    for sp in sps:
        for c in range(sp.nchan):
            tabs_f.append(sp.f[c]); tabs_fp.append(sp.fp[c]); tab_off.append(o)
            o += sp.nknots
    arrays = {
        "cell.f64": (s.cell, np.float64), "pos.f64": (s.pos, np.float64), "species.i32": (s.species, np.int32),
        "sp_rcut.f64": ([sp.rcut for sp in sps], np.float64), "sp_dr.f64": ([sp.dr for sp in sps], np.float64),
        "sp_rs.f64": ([sp.rs for sp in sps], np.float64), "sp_nknots.i32": ([sp.nknots for sp in sps], np.int32),
        "sp_cutoff.i32": ([1 if sp.cutoff else 0 for sp in sps], np.int32), "sp_chan_off.i32": (chan_off, np.int32),
        "chan_l.i32": (np.concatenate([sp.ls for sp in sps]), np.int32),
        "chan_alpha.f64": (np.concatenate([sp.alphas for sp in sps]), np.float64),
        "chan_tab_off.i64": (tab_off, np.int64), "tab_f.f64": (np.concatenate(tabs_f), np.float64),
        "tab_fp.f64": (np.concatenate(tabs_fp), np.float64), "grid.i32": (s.grid, np.int32),
        "blk_i.i32": (s.blk_i, np.int32), "blk_j.i32": (s.blk_j, np.int32), "blk_r.i32": (s.blk_r, np.int32),
        "blk_off.i64": (s.blk_off, np.int64), "v.f64": (s.v, np.float64), "d.f64": (s.d, np.float64),
    }
    for name, (a, dt) in arrays.items():
        np.ascontiguousarray(np.asarray(a), dtype=dt).tofile(os.path.join(d, name))
    with open(os.path.join(d, "meta.txt"), "w") as f:
        f.write(f"{s.natom} {len(sps)} {len(s.blk_i)} {s.ngrid} {s.nnz} {int(chan_off[-1])} {o} 0\n")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV, **kw)
    report = r.stdout + r.stderr
    assert "runtime error" not in report and "AddressSanitizer" not in report and "LeakSanitizer" not in report, report
    assert r.returncode == 0, report
    return report


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    odrv, pdrv = str(d / "oracle_driver"), str(d / "plan_driver")
    run(["gcc", *SAN, "-fopenmp", "-std=c11", "-I", os.path.join(ROOT, "oracle"),
         os.path.join(NATIVE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "gint_oracle.c"), "-lm", "-o", odrv])
    csrc = os.path.join(ROOT, "paper_2409_09399_amd", "csrc")
    run(["g++", *SAN, "-std=c++17", "-pthread", "-I", os.path.join(ROOT, "include"), "-I", csrc,
         os.path.join(NATIVE, "plan_driver.cpp"), os.path.join(csrc, "gint_plan.cpp"), "-o", pdrv])
    return odrv, pdrv


def _three_species():
    from paper_2409_09399_amd import inputs as I
    rng = np.random.default_rng(7)
    sps = [I.make_species("X", "spd", 4.1, 0.01, rng), I.make_species("Y", "sp", 3.3, 0.02, rng),
           I.make_species("Z", "2s2p1d", 5.0, 0.01, rng)]
    cell = np.array([[5.1, 0.0, 0.0], [1.2, 4.6, 0.0], [0.4, -0.7, 5.5]])
    pos = rng.uniform(0, 1, size=(5, 3)) @ cell
    grid = (13, 10, 11)
    v = rng.uniform(-1, 1, size=int(np.prod(grid)))
    return I.assemble(cell, pos, np.array([0, 1, 2, 1, 0]), sps, grid, v, rng, name="san5")


def test_oracle_under_sanitizers(drivers, tmp_path, oracle_mod):
    """Every oracle sum over a whole (small, skewed, three-species) system
    runs clean under ASan/UBSan and reproduces the library build's results."""
    odrv, _ = drivers
    s = _three_species()
    dump(s, str(tmp_path))
    out = run([odrv, str(tmp_path)])
    print(out.strip())
    o = oracle_mod.Oracle(s)
    F, Z, E, _ = o.force_stress()

    def get(name, n):
        return np.fromfile(os.path.join(tmp_path, name), dtype=np.float64, count=n)
    for got, ref in ((get("out_h.f64", s.nnz), o.vlocal()), (get("out_rho.f64", s.ngrid), o.rho()),
                     (get("out_rho_abs.f64", s.ngrid), o.rho_abs()), (get("out_force.f64", 3 * s.natom), F.ravel()),
                     (get("out_z.f64", 9), np.asarray(Z).ravel()), (get("out_e.f64", 1), [E]),
                     (get("out_work.f64", 1), [o.work()])):
        ref = np.asarray(ref, dtype=np.float64)
        assert np.abs(got - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1e-300)


@pytest.mark.parametrize("case", [((0, 0, 0), 0, 1), ((1, 1, 1), 4, 1), ((3, 1, 2), 3, 3), ((0, 0, 0), 6, 1),
                                  ((0, 0, 0), 0, 5), ((0, 0, 0), 8, 7)],
                         ids=["default", "1x1x1_cl4", "3x1x2_cl3_slabs3", "cl6", "slabs5", "cl8_slabs7"])
def test_plan_builder_under_sanitizers(drivers, tmp_path, case):
    """The plan builder runs clean under ASan/UBSan on a skewed three-species
    cell with a ragged grid and on a 76-atom twisted bilayer, its bricks pass
    the brute-force union and pair-table checks, its cluster pairs (clusters
    of up to 4 by default, 3, 6 and 8) store every overlapping pattern block
    exactly once, and the plans of grid slabs along a1 (the streaming
    pipeline's) partition the whole plan's visits and bricks."""
    from paper_2409_09399_amd import inputs as I
    _, pdrv = drivers
    brick, cl, slabs = case
    for k, s in enumerate((_three_species(), I.tbg_system(2, h=0.44))):
        d = tmp_path / f"s{k}"
        d.mkdir()
        dump(s, str(d))
        args = [pdrv, str(d), "brick=%d,%d,%d" % brick, f"cl={cl}", f"slabs={slabs}"]
        out = run(args, timeout=600)
        print(s.name, out.strip())
        assert "plan driver ok" in out
