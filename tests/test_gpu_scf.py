"""One SCF step at the Gamma point on the device (include/gint_scf.h),
through the C ABI, against the oracle's reference step: the oracle's H(R)
and S(R) = H[V = 1], folded over R, solved with scipy.linalg.eigh (a library
routine) and filled by the same rule.  Eigenvalues to 1e-10 of their range;
D(R) to 1e-9 where the occupied subspace is well separated; and the new D
puts exactly n_electrons on the grid (gint_rho, N_e = sum_g w rho_g)."""
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


def scf_step(torch, dev, G, s, nel, kT):
    plan = G.Plan(s)
    v = torch.tensor(s.v, device=dev)
    ones = torch.ones(s.ngrid, dtype=torch.float64, device=dev)
    h = torch.empty(s.nnz, dtype=torch.float64, device=dev)
    sv = torch.empty(s.nnz, dtype=torch.float64, device=dev)
    G.gint_vlocal(plan, v, h)
    G.gint_vlocal(plan, ones, sv)
    scf = G.Scf(plan)
    n = scf.n
    eig = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
    occ = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
    d = torch.full((s.nnz,), np.nan, dtype=torch.float64, device=dev)
    info = torch.full((1,), -7, dtype=torch.int32, device=dev)
    scf.solve(h, sv, nel, kT, eig, occ, d, info)
    rho = torch.empty(s.ngrid, dtype=torch.float64, device=dev)
    ne = torch.empty(1, dtype=torch.float64, device=dev)
    G.gint_rho(plan, d, rho, ne)
    torch.cuda.synchronize()
    out = dict(eig=eig.cpu().numpy(), occ=occ.cpu().numpy(), d=d.cpu().numpy(), info=int(info.cpu()[0]),
               ne=float(ne.cpu()[0]), h=h.cpu().numpy(), s=sv.cpu().numpy())
    scf.close()
    plan.close()
    return out


@pytest.mark.parametrize("case", [("diamond", 0.0), ("diamond", 0.02), ("tbg76", 0.0)],
                         ids=["diamond_aufbau", "diamond_fermi", "tbg76_aufbau"])
def test_scf_step_against_oracle(env, oracle_mod, case):
    torch, dev, G, I = env
    name, kT = case
    s = I.diamond8(0, grid=(24, 24, 24)) if name == "diamond" else I.tbg_system(2, h=0.3)
    nel = 4.0 * s.natom - (1.0 if kT > 0 else 0.0)      # valence electrons of C (one removed: a partly filled level)
    print(f"[gpu] scf step {s.name} n_atoms={s.natom} grid={tuple(int(x) for x in s.grid)} nel={nel} kT={kT}",
          flush=True)
    g = scf_step(torch, dev, G, s, nel, kT)
    assert g["info"] == 0
    o = oracle_mod.Oracle(s)
    h_or, s_or = o.vlocal(), o.vlocal(np.ones(s.ngrid))
    e, f, Z, D = o.scf_gamma(h_or, s_or, nel, kT)
    span = float(np.abs(e).max())
    de = float(np.abs(g["eig"] - e).max())
    print(f"[gpu] scf eigenvalues: n={e.size} max|de|={de:.3e} (range {span:.3e}); "
          f"N_e={g['ne']:.15f}", flush=True)
    assert de <= 1e-10 * span
    assert np.abs(g["occ"] - f).max() <= 1e-9
    assert abs(g["occ"].sum() - nel) <= 1e-10 * nel
    # D is unique when the occupations do not split a (near-)degenerate level
    k = int(np.searchsorted(np.cumsum(f), nel - 1e-9))
    gap = float(e[min(k + 1, e.size - 1)] - e[k]) if k + 1 < e.size else 1.0
    if kT > 0 or gap > 1e-6:
        assert np.abs(g["d"] - D).max() <= 1e-9 * np.abs(D).max(), gap
    # the new D carries exactly n_electrons: N_e = sum_g w rho_g = <D, S> = sum f
    assert abs(g["ne"] - nel) <= 1e-9 * nel
    assert abs(float(np.dot(g["d"], g["s"])) - nel) <= 1e-9 * nel


def test_scf_fold_gamma_matches_oracle(env, oracle_mod):
    torch, dev, G, I = env
    s = I.diamond8(1, grid=(16, 16, 16))
    plan = G.Plan(s)
    scf = G.Scf(plan)
    vals = torch.tensor(np.random.default_rng(5).standard_normal(s.nnz), device=dev)
    dense = torch.full((scf.n * scf.n,), np.nan, dtype=torch.float64, device=dev)
    scf.fold_gamma(vals, dense)
    torch.cuda.synchronize()
    ref = oracle_mod.Oracle(s).fold_gamma(vals.cpu().numpy())
    got = dense.cpu().numpy().reshape(scf.n, scf.n).T      # column-major
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    scf.close()
    plan.close()


def test_scf_loop_keeps_electron_count(env):
    """A few steps of a model self-consistent loop on the device: V_in =
    V_ext + a rho_out with linear mixing; every step's D carries n_electrons."""
    torch, dev, G, I = env
    s = I.diamond8(2, grid=(16, 16, 16))
    plan = G.Plan(s)
    scf = G.Scf(plan)
    vext = torch.tensor(s.v, device=dev)
    ones = torch.ones(s.ngrid, dtype=torch.float64, device=dev)
    sv = torch.empty(s.nnz, dtype=torch.float64, device=dev)
    G.gint_vlocal(plan, ones, sv)
    h = torch.empty(s.nnz, dtype=torch.float64, device=dev)
    d = torch.empty(s.nnz, dtype=torch.float64, device=dev)
    eig = torch.empty(scf.n, dtype=torch.float64, device=dev)
    occ = torch.empty(scf.n, dtype=torch.float64, device=dev)
    rho = torch.zeros(s.ngrid, dtype=torch.float64, device=dev)
    ne = torch.empty(1, dtype=torch.float64, device=dev)
    nel = 32.0
    v = vext.clone()
    for it in range(4):
        G.gint_vlocal(plan, v, h)
        scf.solve(h, sv, nel, 0.01, eig, occ, d)
        G.gint_rho(plan, d, rho, ne)
        v = 0.5 * v + 0.5 * (vext + 0.3 * rho)
        torch.cuda.synchronize()
        print(f"[gpu] scf loop it={it} N_e={float(ne.cpu()[0]):.15f} e_min={float(eig.cpu()[0]):.10f}", flush=True)
        assert abs(float(ne.cpu()[0]) - nel) <= 1e-9 * nel
    scf.close()
    plan.close()
