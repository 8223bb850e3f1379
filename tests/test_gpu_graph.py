"""HIP graph replay and the autotuner (through the C ABI).

A captured step must reproduce the eager calls on every replay, with eager
work and synchronisations between replays, and its outputs poisoned before
each replay so that stale values cannot pass.  Replays are compared with the
eager result to 1e-13 (FP64 atomics may sum in another order) and the eager
result with the oracle to 1e-11.  The autotuner's choice must give the same
results as the defaults.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_09399_amd import gint as G
    return torch, torch.device("cuda:0"), G


def buffers(torch, dev, plan, systems):
    n = plan.n_sys
    b = dict(v=torch.tensor(np.concatenate([s.v for s in systems]), device=dev),
             d=torch.tensor(np.concatenate([s.d for s in systems]), device=dev),
             h=torch.empty(plan.nnz, dtype=torch.float64, device=dev),
             rho=torch.empty(plan.ngrid, dtype=torch.float64, device=dev),
             ne=torch.empty(n, dtype=torch.float64, device=dev),
             F=torch.empty(3 * plan.natom, dtype=torch.float64, device=dev),
             sig=torch.empty(9 * n, dtype=torch.float64, device=dev),
             E=torch.empty(n, dtype=torch.float64, device=dev))
    return b


OUTS = ("h", "rho", "ne", "F", "sig", "E")


def eager(G, plan, b):
    G.gint_vlocal(plan, b["v"], b["h"])
    G.gint_rho(plan, b["d"], b["rho"], b["ne"])
    G.gint_force_stress(plan, b["v"], b["d"], b["F"], b["sig"], b["E"])


def snapshot(torch, b):
    torch.cuda.synchronize()
    return {k: b[k].cpu().numpy().copy() for k in OUTS}


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp16x3"])
def test_graph_replays_match_eager(env, prec):
    torch, dev, G = env
    from paper_2409_09399_amd import inputs as I
    systems = [I.diamond8(0), I.random_molecular_crystal(3, natom=40), I.diamond8(2, grid=(30, 27, 33))]
    print(f"[gpu] graph replay prec={prec} on {[s.name for s in systems]}", flush=True)
    plan = G.Plan(systems, precision=prec)
    b = buffers(torch, dev, plan, systems)
    eager(G, plan, b)
    ref = snapshot(torch, b)
    g = G.Graph(plan, v_loc=b["v"], d_vals=b["d"], h_vals=b["h"], rho=b["rho"], n_elec=b["ne"], force=b["F"],
                stress=b["sig"], energy=b["E"])
    scratch = torch.empty(plan.nnz, dtype=torch.float64, device=dev)
    for rep in range(4):
        for k in OUTS:
            b[k].fill_(float("nan"))
        g.launch()
        got = snapshot(torch, b)
        for k in OUTS:
            assert np.isfinite(got[k]).all(), (rep, k)
            assert rel(got[k], ref[k]) <= 1e-13, (rep, k, rel(got[k], ref[k]))
        # eager work on the same plan and stream between replays
        G.gint_vlocal(plan, b["v"], scratch)
        torch.cuda.synchronize()
        assert rel(scratch.cpu().numpy(), ref["h"]) <= 1e-13
    g.close()
    plan.close()


def test_graph_partial_stages(env):
    """A graph of rho alone leaves the other outputs untouched."""
    torch, dev, G = env
    from paper_2409_09399_amd import inputs as I
    s = I.diamond8(1)
    plan = G.Plan(s)
    b = buffers(torch, dev, plan, [s])
    eager(G, plan, b)
    ref = snapshot(torch, b)
    b["h"].fill_(7.0)
    b["rho"].fill_(float("nan"))
    g = G.Graph(plan, d_vals=b["d"], rho=b["rho"])
    for _ in range(2):
        g.launch()
        torch.cuda.synchronize()
        assert rel(b["rho"].cpu().numpy(), ref["rho"]) <= 1e-13
    assert bool((b["h"] == 7.0).all())
    g.close()
    plan.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp16x3"])
def test_autotune_choice_is_correct(env, oracle_mod, prec):
    """The tuner's choices are the fastest trials of their stages; every
    candidate it timed gives the oracle's result (FP64 to 1e-11; FP16x3 to
    its rho and H bounds), i.e. the tile shape changes the time, not the
    answer; a second call with the same workload returns the cached choice."""
    torch, dev, G = env
    from paper_2409_09399_amd import inputs as I
    s = I.diamond8(0)
    G.autotune_forget()
    opts, rep = G.autotune(s, precision=prec, budget_seconds=30.0)
    print(f"[gpu] autotune {opts} {rep}", flush=True)
    assert not rep["cached"]
    assert len(rep["trials"]) == 8          # the whole candidate list fits the budget here
    assert 1 <= len(rep["trials"]) <= G.GINT_TUNE_MAX
    assert all(t["vlocal_ms"] > 0 and t["rho_force_ms"] > 0 for t in rep["trials"])
    best = rep["trials"][rep["best"]]
    assert best["vlocal_ms"] == min(t["vlocal_ms"] for t in rep["trials"])
    assert opts["cluster_atoms"] == best["cluster_atoms"]
    bb = rep["trials"][rep["best_brick"]]
    assert bb["rho_force_ms"] == min(t["rho_force_ms"] for t in rep["trials"])
    assert tuple(opts["brick"]) == tuple(bb["brick"])
    if prec == 0:
        assert tuple(opts["brick"]) == (0, 0, 0)
    o = oracle_mod.Oracle(s)
    h_ref, rho_ref = o.vlocal(), o.rho()
    tol = 1e-11 if prec == 0 else 1e-6
    cands = [dict(cluster_atoms=t["cluster_atoms"], max_bigcells_per_item=t["max_bigcells_per_item"],
                  brick=tuple(t["brick"]), precision=prec) for t in rep["trials"]]
    for c in [dict(opts)] + cands:
        c.pop("decomposition", None)
        plan = G.Plan(s, **c)
        b = buffers(torch, dev, plan, [s])
        eager(G, plan, b)
        got = snapshot(torch, b)
        eh, er = rel(got["h"], h_ref), rel(got["rho"], rho_ref)
        print(f"[gpu] candidate {c}: H {eh:.2e} rho {er:.2e}", flush=True)
        assert eh <= tol and er <= tol, c
        plan.close()
    opts2, rep2 = G.autotune(s, precision=prec, budget_seconds=30.0)
    assert rep2["cached"] and opts2 == opts and rep2["best"] == rep["best"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp16x3"])
def test_rejected_calls_leave_outputs_untouched(env, prec):
    """The header's error contract, through the raw C ABI: a call rejected
    with GINT_EINVAL (a null argument) enqueues nothing, so outputs it was
    given keep their contents, and the next valid call still works."""
    torch, dev, G = env
    from paper_2409_09399_amd import inputs as I
    s = I.diamond8(2)
    plan = G.Plan(s, precision=prec)
    b = buffers(torch, dev, plan, [s])
    for k in ("h", "rho", "F", "sig", "E", "ne"):
        b[k].fill_(7.0)
    torch.cuda.synchronize()
    lib, p = G._lib, plan._p
    ptr = lambda t: t.data_ptr()
    st = torch.cuda.current_stream().cuda_stream
    assert lib.gint_vlocal(p, None, ptr(b["h"]), st) == G.GINT_EINVAL
    assert lib.gint_rho(p, None, ptr(b["rho"]), ptr(b["ne"]), st) == G.GINT_EINVAL
    assert lib.gint_force_stress(p, ptr(b["v"]), ptr(b["d"]), ptr(b["F"]), None, ptr(b["E"]), st) == G.GINT_EINVAL
    assert lib.gint_rho_force_stress(p, ptr(b["v"]), None, ptr(b["rho"]), ptr(b["ne"]), ptr(b["F"]), ptr(b["sig"]),
                                     ptr(b["E"]), st) == G.GINT_EINVAL
    torch.cuda.synchronize()
    for k in ("h", "rho", "F", "sig", "E", "ne"):
        assert bool((b[k] == 7.0).all()), k
    eager(G, plan, b)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(b["h"]).all()) and not bool((b["h"] == 7.0).all())
    plan.close()
