"""The two tile-store layouts of the mixed Vlocal give the same H.

With one orbital layout over all species the FP16 kernel is built for that
layout: two lanes of a pair of points exchange their converted orbital
pairs and store 32-bit words, and a lane whose partner reaches the bigcell
evaluates with weight 0.  Adding an unused species of another layout to the
same system (its tables scaled down, so that the operand scale stays the
same) selects the per-species instance, which stores each lane's 16-bit
values itself.  Both contract the same operands, so H agrees to the
rounding of the FP64 geometry and sums, which the compiler may contract
differently in the two instances (asserted: 1e-10 of max|H|, four orders
below the form's own error), including the points just outside a cutoff
sphere where only the partner lane is active.  Checked on the jittered
diamond cell and on a 148-atom twisted bilayer on a coarse grid.
"""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def vlocal(G, torch, dev, s):
    plan = G.Plan(s, precision=G.GINT_MIXED_FP16X3)
    v = torch.tensor(s.v, device=dev)
    h = torch.full((s.nnz,), float("nan"), dtype=torch.float64, device=dev)
    G.gint_vlocal(plan, v, h)
    torch.cuda.synchronize()
    plan.close()
    return h.cpu().numpy()


@pytest.mark.parametrize("system", ["diamond", "tbg148"])
def test_paired_and_plain_tile_stores_agree(system):
    import torch
    assert torch.cuda.is_available()
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I
    dev = torch.device("cuda:0")
    s = I.make_config(1) if system == "diamond" else I.tbg_system(3, h=0.44)
    rng = np.random.default_rng(7)
    extra = I.make_species("H", "2s1p", 6.0, 0.01, rng)
    # tables scaled down so that the plan-wide operand scale (a power of two
    # from the largest |phi| over the species) stays that of the carbon
    extra = dataclasses.replace(extra, f=extra.f * 1e-3, fp=extra.fp * 1e-3)
    s2 = dataclasses.replace(s, species_list=list(s.species_list) + [extra])
    print(f"[gpu] store layouts {system}: {s.natom} atoms, grid {tuple(int(x) for x in s.grid)}", flush=True)
    h1 = vlocal(G, torch, dev, s)
    h2 = vlocal(G, torch, dev, s2)
    assert np.all(np.isfinite(h1)) and np.all(np.isfinite(h2))
    scale = float(np.abs(h1).max())
    diff = float(np.abs(h1 - h2).max())
    print(f"[gpu] store layouts {system}: max|H| {scale:.3e}, max|dH| {diff:.3e}", flush=True)
    assert diff <= 1e-10 * scale
