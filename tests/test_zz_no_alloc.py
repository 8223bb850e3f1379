"""gint_energy_noalloc (the entry point that allocates nothing; its partial
sums live in the library's static device scratch) against gint_energy, whose
partial sums live in the plan's workspace: the same two-pass reduction in the
same order, so the results must agree bit for bit.  Two calls in a row, the
second on a smaller plan (fewer systems, fewer points), so that the second
call runs on scratch left over from the first; then a plan with more systems
than the scratch holds is rejected before anything is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I
    return torch, torch.device("cuda:0"), G, I


def energies(torch, dev, G, plan, systems):
    v = torch.tensor(np.concatenate([s.v for s in systems]), device=dev)
    d = torch.tensor(np.concatenate([s.d for s in systems]), device=dev)
    rho = torch.empty(plan.ngrid, dtype=torch.float64, device=dev)
    G.gint_rho(plan, d, rho)
    e_ref = torch.full((plan.n_sys,), np.nan, dtype=torch.float64, device=dev)
    e_new = torch.full((plan.n_sys,), np.nan, dtype=torch.float64, device=dev)
    G.gint_energy(plan, v, rho, e_ref)
    G.gint_energy_noalloc(plan, v, rho, e_new)
    torch.cuda.synchronize()
    # independent check of the value itself: w sum_g V_g rho_g per system
    r, vv = rho.cpu().numpy(), v.cpu().numpy()
    off, host = 0, []
    for s in systems:
        host.append(s.volume / s.ngrid * float(np.dot(vv[off:off + s.ngrid], r[off:off + s.ngrid])))
        off += s.ngrid
    return e_ref.cpu().numpy(), e_new.cpu().numpy(), np.array(host)


def test_noalloc_energy_matches_plan_workspace_form(env):
    torch, dev, G, I = env
    big = [I.diamond8(0, grid=(24, 24, 24)), I.diamond8(1, grid=(20, 20, 20)), I.diamond8(2, grid=(16, 16, 16))]
    small = [I.diamond8(3, grid=(12, 12, 12))]
    for name, systems in (("3 systems", big), ("1 smaller system", small)):
        print(f"[gpu] energy_noalloc on {name}: grids {[tuple(int(x) for x in s.grid) for s in systems]}",
              flush=True)
        plan = G.Plan(systems if len(systems) > 1 else systems[0])
        e_ref, e_new, host = energies(torch, dev, G, plan, systems)
        plan.close()
        assert np.all(np.isfinite(e_new))
        assert np.array_equal(e_ref, e_new), (e_ref, e_new)
        assert np.allclose(e_new, host, rtol=1e-12, atol=0.0)


def test_noalloc_energy_rejects_more_systems_than_scratch(env):
    torch, dev, G, I = env
    # one H-like atom (2s1p) alone in a 20 Bohr cubic cell: one pattern block
    rng = np.random.default_rng(0)
    sp = I.make_species("H", "2s1p", 6.0, 0.01, rng)
    cell = np.eye(3) * 20.0
    s = I.assemble(cell, np.array([[10.0, 10.0, 10.0]]), [0], [sp], (4, 4, 4), np.zeros(64), rng, name="H1")
    n = 513    # 513 x 256 partial sums exceed the 1 MiB scratch
    print(f"[gpu] energy_noalloc rejection: plan of {n} systems", flush=True)
    plan = G.Plan([s] * n)
    v = torch.zeros(plan.ngrid, dtype=torch.float64, device=dev)
    e = torch.full((n,), 7.0, dtype=torch.float64, device=dev)
    with pytest.raises(G.GintError) as ei:
        G.gint_energy_noalloc(plan, v, v, e)
    assert ei.value.code == G.GINT_ENOMEM
    torch.cuda.synchronize()
    assert bool((e == 7.0).all())          # nothing was enqueued
    plan.close()
