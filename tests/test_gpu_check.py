"""gint_check_symmetry: the largest |D_IJR[mu,nu] - D_JI(-R)[nu,mu]| per
system (the symmetry the kernels assume when they use D_sym), through the C
ABI.  The expected values are computed here in FP64 with the same operations,
so the comparison is exact."""
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


def check(G, torch, dev, plan, d):
    out = torch.full((plan.n_sys,), -1.0, dtype=torch.float64, device=dev)
    G.gint_check_symmetry(plan, torch.tensor(d, device=dev), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def transpose_pos(s, b, mu, nu):
    """Element of (J, I, -R) that mirrors (mu, nu) of block b."""
    from paper_2409_09399_amd import inputs as I
    idx = I.block_index(s.blk_i, s.blk_j, s.blk_r)
    i, j, r = int(s.blk_i[b]), int(s.blk_j[b]), s.blk_r[b]
    bt = idx[(j, i, -int(r[0]), -int(r[1]), -int(r[2]))]
    ni = int(s.norb_atom()[i])
    return int(s.blk_off[bt]) + nu * ni + mu


def test_symmetric_and_perturbed(env):
    torch, dev, G, I = env
    s = I.diamond8(1)
    print(f"[gpu] symmetry check {s.name} nblk={len(s.blk_i)}", flush=True)
    plan = G.Plan(s)
    assert check(G, torch, dev, plan, s.d)[0] == 0.0
    norb = s.norb_atom()
    rng = np.random.default_rng(2)
    # an off-diagonal block and a self block (I = J, R = 0), one element each
    self_blk = [b for b in range(len(s.blk_i)) if s.blk_i[b] == s.blk_j[b] and not s.blk_r[b].any()][0]
    other = [b for b in range(len(s.blk_i)) if s.blk_i[b] != s.blk_j[b]][3]
    for b, delta in ((other, 0.25), (self_blk, -3e-9)):
        nj = int(norb[s.blk_j[b]])
        mu, nu = (1, 4) if b == self_blk else (int(rng.integers(norb[s.blk_i[b]])), int(rng.integers(nj)))
        d = s.d.copy()
        k = int(s.blk_off[b]) + mu * nj + nu
        d[k] += delta
        expect = abs(d[k] - d[transpose_pos(s, b, mu, nu)])
        got = check(G, torch, dev, plan, d)[0]
        assert got == expect, (b, got, expect)
    d = s.d.copy()
    d[int(s.blk_off[other])] = np.nan
    assert np.isnan(check(G, torch, dev, plan, d)[0])
    plan.close()


def test_batch_per_system(env):
    """Only the perturbed system of a batched plan reports a difference."""
    torch, dev, G, I = env
    systems = [I.diamond8(1), I.random_molecular_crystal(3, natom=40)]
    plan = G.Plan(systems)
    q = plan.systems[1]
    d = np.concatenate([systems[0].d, systems[1].d])
    s1 = systems[1]
    b = [k for k in range(len(s1.blk_i)) if s1.blk_i[k] != s1.blk_j[k]][0]
    nj = int(s1.norb_atom()[s1.blk_j[b]])
    mu, nu = 0, min(1, nj - 1)
    off = int(q["nnz_off"])
    k = off + int(s1.blk_off[b]) + mu * nj + nu
    d[k] += 1e-6
    got = check(G, torch, dev, plan, d)
    assert got[0] == 0.0
    assert got[1] == abs(d[k] - d[off + transpose_pos(s1, b, mu, nu)])
    plan.close()
