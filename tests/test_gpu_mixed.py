"""Mixed-precision forms against the FP64 oracle (through the C ABI).

GINT_MIXED_FP16X3: FP32 orbitals, FP16 hi+lo split operands with three FP16
MFMA products and FP32 accumulation per bigcell, FP64 across bigcells.
Targets: |H - H_oracle| <= 1e-6 Ha and |F - F_oracle| <= 1e-5 Ha/Bohr; the
rho and stress errors are stated.  rho is bounded point by point against the
magnitude scale of its terms, rho_abs(g) = sum |phi||D||phi| from the oracle:
the split operands carry about 22 bits (2^-22 per product, three products),
phi is evaluated and psi and the per-point dot products are accumulated in
FP32 (at most 64 + 16 terms of 2^-24), which bounds |d rho(g)| by about
5.5e-6 rho_abs(g).  The 16-bit operands are scaled so that the largest |phi|
maps into [2^12, 2^13); values below FP16's normal range (2^-14) keep an
absolute step of 2^-24, an absolute floor of 2^-37 max|phi| per value, which
in the far tails of the orbitals dominates.  The test asserts
|d rho(g)| <= 1e-5 (rho_abs(g) + 1e-10 max rho_abs).  rho itself can be much
smaller than rho_abs by cancellation, so the max-norm relative error is only
recorded.  Stress and energy: relative 1e-5.
GINT_MIXED_BF16X3 (about 16 significant bits per operand: 3 x 2^-16 per
product) is checked against bounds 10x (rho) and 100x (the rest) looser.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def run(G, torch, dev, s, precision, decomposition=0, brick=(0, 0, 0), fused=True, cluster_atoms=0):
    """Vlocal, rho and force/stress of one system; with fused, also the
    one-pass rho + force/stress (out["fused"]), checked by the callers at the
    same bounds (in the mixed forms the two passes round differently)."""
    plan = G.Plan(s, precision=precision, decomposition=decomposition, brick=brick, cluster_atoms=cluster_atoms)
    print(f"[mixed] plan {s.name} prec={precision} decomposition={plan.sizes.decomposition} "
          f"brick={tuple(plan.sizes.brick)} nbricks={plan.sizes.nbricks} clusters={plan.sizes.ncluster}", flush=True)
    v = torch.tensor(s.v, device=dev)
    d = torch.tensor(s.d, device=dev)
    h = torch.full((s.nnz,), float("nan"), dtype=torch.float64, device=dev)
    rho = torch.full((s.ngrid,), float("nan"), dtype=torch.float64, device=dev)
    F = torch.full((s.natom * 3,), float("nan"), dtype=torch.float64, device=dev)
    sig = torch.full((9,), float("nan"), dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    G.gint_vlocal(plan, v, h)
    G.gint_rho(plan, d, rho)
    G.gint_force_stress(plan, v, d, F, sig, E)
    torch.cuda.synchronize()
    out = dict(h=h.cpu().numpy(), rho=rho.cpu().numpy(), F=F.cpu().numpy().reshape(-1, 3),
               sig=sig.cpu().numpy().reshape(3, 3), E=float(E.cpu()[0]))
    if fused:
        rho2 = torch.full((s.ngrid,), float("nan"), dtype=torch.float64, device=dev)
        F2 = torch.full((s.natom * 3,), float("nan"), dtype=torch.float64, device=dev)
        sig2 = torch.full((9,), float("nan"), dtype=torch.float64, device=dev)
        E2 = torch.zeros(1, dtype=torch.float64, device=dev)
        G.gint_rho_force_stress(plan, v, d, rho2, F2, sig2, energy=E2)
        torch.cuda.synchronize()
        out["fused"] = dict(h=out["h"], rho=rho2.cpu().numpy(), F=F2.cpu().numpy().reshape(-1, 3),
                            sig=sig2.cpu().numpy().reshape(3, 3), E=float(E2.cpu()[0]))
    plan.close()
    return out


def rho_scaled(got, ref, ref_abs):
    """max_g |got - ref| / (rho_abs(g) + 1e-10 max rho_abs): the error
    relative to the magnitude of rho's terms at each point, with the absolute
    floor of the scaled 16-bit operands."""
    err = np.abs(np.asarray(got) - np.asarray(ref))
    ra = np.asarray(ref_abs)
    return float(np.max(err / (ra + 1e-10 * ra.max() + 1e-300), initial=0.0))


def errors(gpu, ref):
    e = {}
    e["H_abs"] = float(np.abs(gpu["h"] - ref["h"]).max())
    e["rho_rel"] = float(np.abs(gpu["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max())
    e["rho_pt"] = rho_scaled(gpu["rho"], ref["rho"], ref["rho_abs"])
    e["F_abs"] = float(np.abs(gpu["F"] - ref["F"]).max())
    e["sigma_rel"] = float(np.abs(gpu["sig"] - ref["sig"]).max() / np.abs(ref["sig"]).max())
    e["E_rel"] = abs(gpu["E"] - ref["E"]) / abs(ref["E"])
    return e


BOUNDS = {1: dict(H_abs=1e-6, F_abs=1e-5, rho_pt=1e-5, sigma_rel=1e-5, E_rel=1e-5),
          2: dict(H_abs=1e-4, F_abs=1e-3, rho_pt=1e-4, sigma_rel=1e-3, E_rel=1e-3)}


def record(name, prec, errs):
    d = os.environ.get("GINT_ERROR_LOG")
    if d:
        with open(d, "a") as f:
            f.write(json.dumps({"case": name, "precision": prec, **errs}) + "\n")


# 0: the default (Vlocal on cluster pairs, rho and force on bricks)
DECOMP = [0, 1, 2, 3]
DECOMP_IDS = ["default", "cluster_pairs", "bigcell", "bigcell_rho_force"]


@pytest.mark.parametrize("decomp", DECOMP, ids=DECOMP_IDS)
@pytest.mark.parametrize("prec", [1, 2], ids=["fp16x3", "bf16x3"])
def test_mixed_diamond(torch_dev, oracle_mod, prec, decomp):
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.diamond8(0)
    o = oracle_mod.Oracle(s)
    F, Z, E, sig = o.force_stress()
    ref = dict(h=o.vlocal(), rho=o.rho(), rho_abs=o.rho_abs(), F=F, sig=sig, E=E)
    got = run(G, torch, dev, s, prec, decomposition=decomp)
    errs, errf = errors(got, ref), errors(got["fused"], ref)
    print("[mixed] diamond", prec, decomp, errs, "fused", errf, flush=True)
    record(f"diamond8/{DECOMP_IDS[decomp]}", prec, errs)
    for k, b in BOUNDS[prec].items():
        assert errs[k] <= b, (k, errs[k], b)
        assert errf[k] <= b, ("fused", k, errf[k], b)


@pytest.mark.parametrize("prec", [1, 2], ids=["fp16x3", "bf16x3"])
def test_mixed_tbg868_sampled(torch_dev, oracle_mod, prec):
    """The benchmark workload in mixed precision: sampled rho points, H
    blocks and atom forces from the oracle."""
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.make_config(2)
    gpu = run(G, torch, dev, s, prec)
    o = oracle_mod.Oracle(s)
    rng = np.random.default_rng(1)
    g = rng.choice(s.ngrid, 200, replace=False)
    r_or = o.rho_points(g)
    blks = rng.choice(len(s.blk_i), 16, replace=False)
    herr = 0.0
    for b, ref in zip(blks, o.vlocal_blocks(blks)):
        got = gpu["h"][s.blk_off[b]:s.blk_off[b] + ref.size].reshape(ref.shape)
        herr = max(herr, float(np.abs(got - ref).max()))
    atoms = rng.choice(s.natom, 3, replace=False)
    Fo, _ = o.force_atoms(atoms)
    errs = {"H_abs": herr, "rho_rel": float(np.abs(gpu["rho"][g] - r_or).max() / np.abs(gpu["rho"]).max()),
            "rho_pt": rho_scaled(gpu["rho"][g], r_or, o.rho_abs_points(g)),
            "F_abs": float(np.abs(gpu["F"][atoms] - Fo).max())}
    # every output against the FP64 path on the same workload (itself checked
    # against the oracle in the parity tests): stress and energy included
    f64 = run(G, torch, dev, s, 0)
    full = {"H_abs_all": float(np.abs(gpu["h"] - f64["h"]).max()),
            "F_abs_all": float(np.abs(gpu["F"] - f64["F"]).max()),
            "rho_rel_all": float(np.abs(gpu["rho"] - f64["rho"]).max() / np.abs(f64["rho"]).max()),
            "sigma_rel": float(np.abs(gpu["sig"] - f64["sig"]).max() / np.abs(f64["sig"]).max()),
            "E_rel": abs(gpu["E"] - f64["E"]) / abs(f64["E"])}
    errs.update(full)
    print("[mixed] tbg868", prec, errs, flush=True)
    record("tbg868_sampled", prec, errs)
    for k in ("H_abs", "rho_pt", "F_abs", "sigma_rel", "E_rel"):
        assert errs[k] <= BOUNDS[prec][k], (k, errs[k])
    assert errs["H_abs_all"] <= BOUNDS[prec]["H_abs"] and errs["F_abs_all"] <= BOUNDS[prec]["F_abs"]


def test_tbg148_coarse_full_oracle(torch_dev, oracle_mod):
    """A 148-atom twisted bilayer (commensurate i = 3) on a coarse grid
    (h = 0.44 Bohr) against the full oracle: every output of the FP64 path to
    1e-11 (stress included), and of FP16x3 and BF16x3 to their bounds."""
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.tbg_system(3, h=0.44)
    print(f"[mixed] tbg148 coarse grid {tuple(int(x) for x in s.grid)} natom {s.natom}", flush=True)
    o = oracle_mod.Oracle(s)
    F, Z, E, sig = o.force_stress()
    ref = dict(h=o.vlocal(), rho=o.rho(), rho_abs=o.rho_abs(), F=F, sig=sig, E=E)
    e64 = errors(run(G, torch, dev, s, 0), ref)
    e64["F_rel"] = e64["F_abs"] / float(np.abs(F).max())
    e64["H_rel"] = e64["H_abs"] / float(np.abs(ref["h"]).max())
    print("[mixed] tbg148 fp64", e64, flush=True)
    for k in ("H_rel", "rho_rel", "F_rel", "sigma_rel", "E_rel"):
        assert e64[k] <= 1e-11, (k, e64[k])
    # FP16x3 and BF16x3 on the default plan, and FP16x3 with Vlocal on
    # clusters of eight atoms (the eight-wave kernel: many pairs, split items)
    for prec, cl in ((1, 0), (2, 0), (1, 8)):
        errs = errors(run(G, torch, dev, s, prec, cluster_atoms=cl, fused=False), ref)
        print("[mixed] tbg148", prec, f"cl={cl}", errs, flush=True)
        record(f"tbg148_coarse/cl{cl}", prec, errs)
        for k, b in BOUNDS[prec].items():
            assert errs[k] <= b, (prec, cl, k, errs[k], b)


@pytest.mark.parametrize("case", [(1, (0, 0, 0), 0), (2, (0, 0, 0), 0), (2, (1, 1, 1), 0), (2, (3, 1, 2), 0),
                                  (3, (0, 0, 0), 0), (0, (0, 0, 0), 0), (0, (0, 0, 0), 8), (3, (0, 0, 0), 6)],
                         ids=["cluster_pairs", "bigcell", "bigcell_1x1x1", "bigcell_3x1x2", "bigcell_rho_force",
                              "default", "default_cl8", "bigcell_rho_force_cl6"])
@pytest.mark.parametrize("prec", [1, 2], ids=["fp16x3", "bf16x3"])
def test_mixed_three_species(torch_dev, oracle_mod, prec, case):
    """Species with different channel sets (spd, sp, 2s2p1d) in a skewed cell
    on a grid that is not a multiple of 4 along any axis, against the full
    oracle, at the same bounds; both decompositions, and bricks of several
    shapes."""
    decomp, brick, cl = case
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    rng = np.random.default_rng(7)
    sps = [I.make_species("X", "spd", 4.1, 0.01, rng), I.make_species("Y", "sp", 3.3, 0.02, rng),
           I.make_species("Z", "2s2p1d", 5.0, 0.01, rng)]
    cell = np.array([[5.1, 0.0, 0.0], [1.2, 4.6, 0.0], [0.4, -0.7, 5.5]])
    pos = rng.uniform(0, 1, size=(5, 3)) @ cell
    grid = (21, 18, 22)
    millers = I.random_millers_box(rng, 8, 2)
    v = I.plane_wave_potential(grid, millers, np.full(8, 0.3), rng.uniform(0, 6.28, 8))
    s = I.assemble(cell, pos, np.array([0, 1, 2, 1, 0]), sps, grid, v, rng, name="mixed5")
    o = oracle_mod.Oracle(s)
    F, Z, E, sig = o.force_stress()
    ref = dict(h=o.vlocal(), rho=o.rho(), rho_abs=o.rho_abs(), F=F, sig=sig, E=E)
    got = run(G, torch, dev, s, prec, decomposition=decomp, brick=brick, cluster_atoms=cl)
    errs, errf = errors(got, ref), errors(got["fused"], ref)
    print("[mixed] three species", prec, case, errs, "fused", errf, flush=True)
    record(f"mixed5/{DECOMP_IDS[decomp]}/{brick}/cl{cl}", prec, errs)
    for k, b in BOUNDS[prec].items():
        assert errs[k] <= b, (k, errs[k], b)
        assert errf[k] <= b, ("fused", k, errf[k], b)
