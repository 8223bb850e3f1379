"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bar (plain FP64 path): max-norm relative error ||gpu - oracle||_inf /
||oracle||_inf <= 1e-11 for H, rho, F and sigma; W (an integer count) must
match exactly.  Small cases are compared element by element; the 868-atom
twisted bilayer (the benchmark workload, same plan options as bench.py) is
compared on sampled outputs the oracle computes one by one and on identities
that hold at any size.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def G():
    from paper_2409_09399_amd import gint
    return gint


def run_all(G, torch, dev, s, **plan_kw):
    print(f"[gpu] {s.name} natom={s.natom} grid={tuple(int(x) for x in s.grid)} opts={plan_kw}", flush=True)
    plan = G.Plan(s, **plan_kw)
    v = torch.tensor(s.v, device=dev)
    d = torch.tensor(s.d, device=dev)
    h = torch.full((s.nnz,), float("nan"), dtype=torch.float64, device=dev)
    rho = torch.full((s.ngrid,), float("nan"), dtype=torch.float64, device=dev)
    ne = torch.zeros(1, dtype=torch.float64, device=dev)
    F = torch.full((s.natom * 3,), float("nan"), dtype=torch.float64, device=dev)
    sig = torch.full((9,), float("nan"), dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    W = torch.zeros(1, dtype=torch.float64, device=dev)
    G.gint_vlocal(plan, v, h)
    G.gint_rho(plan, d, rho, ne)
    G.gint_force_stress(plan, v, d, F, sig, E)
    G.gint_work_units(plan, W)
    torch.cuda.synchronize()
    out = dict(h=h.cpu().numpy(), rho=rho.cpu().numpy(), ne=float(ne.cpu()[0]), F=F.cpu().numpy().reshape(-1, 3),
               sig=sig.cpu().numpy().reshape(3, 3), E=float(E.cpu()[0]), W=float(W.cpu()[0]))
    plan.close()
    return out


def full_oracle(oracle_mod, s):
    o = oracle_mod.Oracle(s)
    F, Z, E, sig = o.force_stress()
    rho = o.rho()
    return dict(h=o.vlocal(), rho=rho, ne=float(rho.sum()) * s.volume / s.ngrid, F=F, sig=sig, E=E, W=o.work())


def check_full(gpu, ref):
    errs = {k: rel(gpu[k], ref[k]) for k in ("h", "rho", "F", "sig")}
    errs["E"] = abs(gpu["E"] - ref["E"]) / abs(ref["E"])
    errs["ne"] = abs(gpu["ne"] - ref["ne"]) / abs(ref["ne"])
    print("[gpu] errors", errs, flush=True)
    for k, e in errs.items():
        assert e <= TOL, (k, e)
    assert gpu["W"] == ref["W"]


def test_diamond_config(G, torch_dev, oracle_mod):
    """Jittered 8-atom diamond, 32^3 grid, 13 orbitals/atom, rcut 6."""
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.diamond8(0)
    check_full(run_all(G, torch, dev, s), full_oracle(oracle_mod, s))


def test_ragged_grid_and_cluster_sizes(G, torch_dev, oracle_mod):
    """Grid not divisible by the 4^3 bigcell; every cluster size gives the
    same result; short work items (ragged item tails)."""
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.diamond8(2, grid=(30, 27, 33))
    ref = full_oracle(oracle_mod, s)
    for cl, mb in ((4, 0), (3, 7), (1, 0), (2, 1)):
        check_full(run_all(G, torch, dev, s, cluster_atoms=cl, max_bigcells_per_item=mb), ref)


def test_mixed_species_lmax2(G, torch_dev, oracle_mod):
    """Three species with different channel sets (spd, sp, 2s2p1d), a skewed
    cell and rcut comparable to the cell size."""
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    rng = np.random.default_rng(7)
    sps = [I.make_species("X", "spd", 4.1, 0.01, rng), I.make_species("Y", "sp", 3.3, 0.02, rng),
           I.make_species("Z", "2s2p1d", 5.0, 0.01, rng)]
    cell = np.array([[5.1, 0.0, 0.0], [1.2, 4.6, 0.0], [0.4, -0.7, 5.5]])
    pos = rng.uniform(0, 1, size=(5, 3)) @ cell
    grid = (20, 18, 22)
    millers = I.random_millers_box(rng, 8, 2)
    v = I.plane_wave_potential(grid, millers, np.full(8, 0.3), rng.uniform(0, 6.28, 8))
    s = I.assemble(cell, pos, np.array([0, 1, 2, 1, 0]), sps, grid, v, rng, name="mixed5")
    check_full(run_all(G, torch, dev, s), full_oracle(oracle_mod, s))


def test_single_atom_and_atom_on_grid_point(G, torch_dev, oracle_mod):
    """Degenerate cases: one atom (self pair only), sitting exactly on a grid
    point (r = 0 in the gradient)."""
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    rng = np.random.default_rng(3)
    sp = I.make_species("C", "2s2p1d", 4.0, 0.01, rng)
    cell = np.eye(3) * 9.0
    grid = (24, 24, 24)
    v = I.plane_wave_potential(grid, I.random_millers_box(rng, 6, 2), np.full(6, 0.5), rng.uniform(0, 6, 6))
    s = I.assemble(cell, np.array([[3.0, 4.5, 6.0]]), np.array([0]), [sp], grid, v, rng, name="one_atom")
    check_full(run_all(G, torch, dev, s), full_oracle(oracle_mod, s))


def test_tbg76(G, torch_dev, oracle_mod):
    """Smallest twisted bilayer of the paper's series (76 atoms), coarse grid."""
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.tbg_system(2, grid=(40, 40, 96))
    check_full(run_all(G, torch, dev, s), full_oracle(oracle_mod, s))


@pytest.fixture(scope="module")
def tbg868(G, torch_dev):
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.make_config(2)
    return s, run_all(G, torch, dev, s)


def test_tbg868_sampled(tbg868, oracle_mod):
    """The benchmark workload: 868-atom bilayer, 312 x 312 x 120 grid.
    rho at sampled points, sampled H blocks and forces on sampled atoms are
    computed by the oracle one by one."""
    s, gpu = tbg868
    o = oracle_mod.Oracle(s)
    rng = np.random.default_rng(0)
    g = rng.choice(s.ngrid, 300, replace=False)
    r_or = o.rho_points(g)
    assert rel(gpu["rho"][g], r_or) <= TOL * max(1.0, np.abs(gpu["rho"]).max() / np.abs(r_or).max())
    blks = rng.choice(len(s.blk_i), 24, replace=False)
    hmax = np.abs(gpu["h"]).max()
    for b, ref in zip(blks, o.vlocal_blocks(blks)):
        got = gpu["h"][s.blk_off[b]:s.blk_off[b] + ref.size].reshape(ref.shape)
        assert np.abs(got - ref).max() <= TOL * hmax
    atoms = rng.choice(s.natom, 4, replace=False)
    Fo, Zo = o.force_atoms(atoms)
    assert np.abs(gpu["F"][atoms] - Fo).max() <= TOL * np.abs(gpu["F"]).max()


def test_tbg868_identities(tbg868, oracle_mod):
    """Identities at full size: trace <D,H> = E = sum w V rho; N_e; W."""
    s, gpu = tbg868
    w = s.volume / s.ngrid
    tr = float(np.dot(s.d, gpu["h"]))
    e_rho = float(np.dot(s.v, gpu["rho"])) * w
    assert abs(tr - gpu["E"]) <= 1e-11 * abs(gpu["E"])
    assert abs(e_rho - gpu["E"]) <= 1e-11 * abs(gpu["E"])
    assert abs(gpu["ne"] - float(gpu["rho"].sum()) * w) <= 1e-11 * abs(gpu["ne"])
    assert gpu["W"] == oracle_mod.Oracle(s).work()
    # translation: total force of a constant potential vanishes
    assert np.isfinite(gpu["sig"]).all()


@pytest.mark.parametrize("case", ["diamond", "tbg76", "mixed5"])
def test_fused_rho_force(G, torch_dev, oracle_mod, case):
    """gint_rho_force_stress (one pass over the ordered pairs) gives the same
    rho, N_e, F, sigma and E as the separate calls, to the FP64 bar."""
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    if case == "diamond":
        s = I.diamond8(3)
    elif case == "tbg76":
        s = I.tbg_system(2, grid=(40, 40, 96))
    else:
        rng = np.random.default_rng(7)
        sps = [I.make_species("X", "spd", 4.1, 0.01, rng), I.make_species("Y", "sp", 3.3, 0.02, rng),
               I.make_species("Z", "2s2p1d", 5.0, 0.01, rng)]
        cell = np.array([[5.1, 0.0, 0.0], [1.2, 4.6, 0.0], [0.4, -0.7, 5.5]])
        pos = rng.uniform(0, 1, size=(5, 3)) @ cell
        grid = (20, 18, 22)
        v = I.plane_wave_potential(grid, I.random_millers_box(rng, 8, 2), np.full(8, 0.3), rng.uniform(0, 6.28, 8))
        s = I.assemble(cell, pos, np.array([0, 1, 2, 1, 0]), sps, grid, v, rng, name="mixed5")
    print(f"[gpu] fused rho+force {s.name}", flush=True)
    plan = G.Plan(s)
    v = torch.tensor(s.v, device=dev)
    d = torch.tensor(s.d, device=dev)
    rho = torch.full((s.ngrid,), float("nan"), dtype=torch.float64, device=dev)
    ne = torch.zeros(1, dtype=torch.float64, device=dev)
    F = torch.full((s.natom * 3,), float("nan"), dtype=torch.float64, device=dev)
    sig = torch.full((9,), float("nan"), dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    G.gint_rho_force_stress(plan, v, d, rho, F, sig, n_elec=ne, energy=E)
    torch.cuda.synchronize()
    o = oracle_mod.Oracle(s)
    Fo, Zo, Eo, sigo = o.force_stress()
    rho_o = o.rho()
    assert rel(rho.cpu().numpy(), rho_o) <= TOL
    assert rel(F.cpu().numpy().reshape(-1, 3), Fo) <= TOL
    assert rel(sig.cpu().numpy().reshape(3, 3), sigo) <= TOL
    assert abs(float(E.cpu()[0]) - Eo) <= TOL * abs(Eo)
    ne_o = float(rho_o.sum()) * s.volume / s.ngrid
    assert abs(float(ne.cpu()[0]) - ne_o) <= TOL * abs(ne_o)
    plan.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp16x3"])
def test_layout_instances_agree(G, torch_dev, prec):
    """A plan whose species all have the 2s2p1d channel layout runs kernels
    with that layout built in; adding an unused species of another layout
    (spd) sends the same atoms through the kernels that pick the layout per
    species.  Both give the same H, rho, F, sigma and E (FP64: to round-off
    of the summation order; FP16x3: to its split precision)."""
    import dataclasses
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.diamond8(4)
    extra = I.make_species("X", "spd", 4.0, 0.01, np.random.default_rng(0))
    s2 = dataclasses.replace(s, species_list=list(s.species_list) + [extra], name=s.name + "+unused_spd")
    a = run_all(G, torch, dev, s, precision=prec)
    b = run_all(G, torch, dev, s2, precision=prec)
    tol = 1e-13 if prec == 0 else 1e-6
    for k in ("h", "rho", "F", "sig"):
        assert rel(b[k], a[k]) <= tol, (k, rel(b[k], a[k]))
    assert abs(b["E"] - a["E"]) <= tol * abs(a["E"])
    assert b["W"] == a["W"]
