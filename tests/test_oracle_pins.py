"""Pins of the FP64 oracle to mathematics (no GPU).

The paper prints no values of H, rho, forces or stress, so the oracle is pinned
by results fixed by the mathematics of its definitions (Eq. 1-5):
  * closed-form overlaps, forces and strain derivatives of uncut s/p Gaussians
    with V = 1 (Gaussian product theorem; the grid sum equals the integral up
    to aliasing exp(-pi^2/(p h^2)) ~ e^-60);
  * the adjoint/trace identity sum<D,H> = sum_g w V rho and the electron count;
  * the symmetry H_JI(-R) = H_IJR^T;
  * brute-force enumeration on tiny inputs and a dense-matrix product;
  * invariances (grid translation, atom permutation, linearity);
  * central finite differences of the energy for forces and strain;
  * the Hermite interpolant's error bound, Y_lm orthonormality, the addition
    theorem and the gradient of the orbitals.
"""
import math

import numpy as np
import pytest

from paper_2409_09399_amd import inputs as I

C0 = 1.0 / (2.0 * math.sqrt(math.pi))
C1 = math.sqrt(3.0 / (4.0 * math.pi))
# p orbitals m = -1, 0, 1 are the y, z, x components
PCOMP = (1, 2, 0)


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------

def _gauss_system(grid=(40, 40, 40), L=8.0):
    rng = np.random.default_rng(11)
    rc1 = math.sqrt(41.5 / 1.1)
    rc2 = math.sqrt(41.5 / 1.0)
    sp1 = I.make_species("A", "sp", rc1, 0.01, rng, alphas=[1.1, 1.7], cutoff=False)
    sp2 = I.make_species("B", "sp", rc2, 0.01, rng, alphas=[1.9, 1.0], cutoff=False)
    cell = np.array([[L, 0, 0], [0.6, L, 0], [0.3, -0.4, L]])
    pos = np.array([[1.13, 2.31, 0.72], [2.41, 3.13, 1.92], [3.1, 1.4, 2.3]])
    v = np.ones(int(np.prod(grid)))
    return I.assemble(cell, pos, np.array([0, 1, 1]), [sp1, sp2], grid, v, rng)


def _overlap_block(sys, blk, A, Bp):
    """Closed-form <phi_I,mu | phi_J,nu> (integral over all space) for uncut
    s/p Gaussians centred at A and Bp; works for complex centres."""
    spI = sys.species_list[sys.species[sys.blk_i[blk]]]
    spJ = sys.species_list[sys.species[sys.blk_j[blk]]]

    def orbs(sp):
        out = []
        for c, l in enumerate(sp.ls):
            for m in range(2 * l + 1):
                out.append((int(l), m, float(sp.alphas[c])))
        return out

    oi, oj = orbs(spI), orbs(spJ)
    S = np.zeros((len(oi), len(oj)), dtype=complex)
    for mu, (li, mi, a) in enumerate(oi):
        for nu, (lj, mj, b) in enumerate(oj):
            p = a + b
            P = (a * A + b * Bp) / p
            dd = A - Bp
            G = (math.pi / p) ** 1.5 * np.exp(-a * b * np.sum(dd * dd) / p)
            if li == 0 and lj == 0:
                val = C0 * C0 * G
            elif li == 0 and lj == 1:
                val = C0 * C1 * (P - Bp)[PCOMP[mj]] * G
            elif li == 1 and lj == 0:
                val = C1 * C0 * (P - A)[PCOMP[mi]] * G
            else:
                i, j = PCOMP[mi], PCOMP[mj]
                val = C1 * C1 * ((P - A)[i] * (P - Bp)[j] + (1.0 / (2.0 * p) if i == j else 0.0)) * G
            S[mu, nu] = val
    return S


def _closed_energy(sys, pos, cell):
    """E = sum over blocks <D, S> with closed-form S (V = 1)."""
    norb = sys.norb_atom()
    E = 0.0
    for k in range(len(sys.blk_i)):
        i, j = sys.blk_i[k], sys.blk_j[k]
        A = pos[i]
        Bp = pos[j] + sys.blk_r[k] @ cell
        S = _overlap_block(sys, k, A, Bp)
        ni, nj = int(norb[i]), int(norb[j])
        D = sys.d[sys.blk_off[k]:sys.blk_off[k] + ni * nj].reshape(ni, nj)
        E = E + np.sum(D * S)
    return E


@pytest.fixture(scope="module")
def gauss(oracle_mod):
    s = _gauss_system()
    return s, oracle_mod.Oracle(s, radial="analytic")


def test_closed_form_overlaps(gauss):
    """H[V=1] equals the Gaussian-product overlaps block by block."""
    s, o = gauss
    h = o.vlocal()
    norb = s.norb_atom()
    err, ref = 0.0, 0.0
    for k in range(len(s.blk_i)):
        i, j = s.blk_i[k], s.blk_j[k]
        S = _overlap_block(s, k, s.pos[i], s.pos[j] + s.blk_r[k] @ s.cell).real
        ni, nj = int(norb[i]), int(norb[j])
        Hk = h[s.blk_off[k]:s.blk_off[k] + ni * nj].reshape(ni, nj)
        err = max(err, np.abs(Hk - S).max())
        ref = max(ref, np.abs(S).max())
    assert err / ref < 1e-12, err / ref


def test_closed_form_electron_count(gauss):
    s, o = gauss
    rho = o.rho()
    w = s.volume / s.ngrid
    ne = np.sum(rho) * w
    ref = _closed_energy(s, s.pos, s.cell).real
    assert abs(ne - ref) < 1e-12 * max(1.0, abs(ref))


def test_closed_form_force(gauss):
    """F_K = -dE/dtau_K from the closed form (complex-step derivative)."""
    s, o = gauss
    F, Z, E, sig = o.force_stress()
    h = 1e-30
    Fref = np.zeros_like(F)
    for K in range(s.natom):
        for a in range(3):
            pos = s.pos.astype(complex)
            pos[K, a] += 1j * h
            Fref[K, a] = -_closed_energy(s, pos, s.cell).imag / h
    assert np.abs(F - Fref).max() < 1e-11 * np.abs(Fref).max()
    assert abs(E - _closed_energy(s, s.pos, s.cell).real) < 1e-12


def test_closed_form_strain_derivative(gauss):
    """Z_ab = dE/d eps_ab at fixed w: E(eps) = sum <D, S((1+eps) d)> / det(1+eps)."""
    s, o = gauss
    F, Z, E, sig = o.force_stress()
    h = 1e-30
    Zref = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3), dtype=complex)
            eps[a, b] = 1j * h
            M = np.eye(3) + eps
            Es = _closed_energy(s, s.pos @ M.T, s.cell @ M.T) / np.linalg.det(M)
            Zref[a, b] = Es.imag / h
    assert np.abs(Z - Zref).max() < 1e-11 * np.abs(Zref).max()
    assert np.allclose(sig, -Z / s.volume)


# ----------------------------------------------------------------------------
# identities on the table-mode workload
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def diamond(oracle_mod):
    s = I.diamond8(0)
    o = oracle_mod.Oracle(s)
    return s, o, o.vlocal(), o.rho(), o.force_stress()


def test_trace_identity(diamond):
    """sum_IJR <D_IJR, H_IJR> = sum_g w V_g rho_g (Vlocal is the adjoint of rho)."""
    s, o, h, rho, fs = diamond
    lhs = float(np.dot(s.d, h))
    rhs = float(np.dot(s.v, rho)) * s.volume / s.ngrid
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert abs(fs[2] - rhs) < 1e-12 * abs(rhs)


def test_electron_count_identity(diamond, oracle_mod):
    s, o, h, rho, fs = diamond
    h1 = o.vlocal(v=np.ones(s.ngrid))
    ne = rho.sum() * s.volume / s.ngrid
    assert abs(ne - float(np.dot(s.d, h1))) < 1e-12 * abs(ne)


def test_h_symmetry(diamond):
    s, o, h, rho, fs = diamond
    idx = I.block_index(s.blk_i, s.blk_j, s.blk_r)
    n = 13
    for k in range(len(s.blk_i)):
        i, j, r = int(s.blk_i[k]), int(s.blk_j[k]), s.blk_r[k]
        kt = idx[(j, i, -int(r[0]), -int(r[1]), -int(r[2]))]
        a = h[s.blk_off[k]:s.blk_off[k] + n * n].reshape(n, n)
        b = h[s.blk_off[kt]:s.blk_off[kt] + n * n].reshape(n, n)
        assert np.abs(a - b.T).max() < 1e-14


def test_force_sum_matches_translation(diamond):
    """Shifting every atom by t changes E only through V: with V = const the
    total force vanishes (translation invariance of the overlaps)."""
    s, o, h, rho, fs = diamond
    F, Z, E, sig = o.force_stress(v=np.full(s.ngrid, 0.7))
    assert np.abs(F.sum(0)).max() < 1e-6 * np.abs(F).max()


def test_sampled_match_full(diamond):
    s, o, h, rho, fs = diamond
    rng = np.random.default_rng(5)
    g = rng.choice(s.ngrid, 50, replace=False)
    assert np.abs(o.rho_points(g) - rho[g]).max() < 1e-13
    ra = o.rho_abs()
    assert np.abs(o.rho_abs_points(g) - ra[g]).max() < 1e-13 * ra.max()
    assert np.all(ra >= np.abs(rho) * (1 - 1e-14))
    blks = rng.choice(len(s.blk_i), 12, replace=False)
    for b, blk in zip(blks, o.vlocal_blocks(blks)):
        ref = h[s.blk_off[b]:s.blk_off[b] + blk.size].reshape(blk.shape)
        assert np.abs(blk - ref).max() < 1e-14
    F, Z, E, sig = fs
    Fs, Zs = o.force_atoms(np.arange(s.natom))
    assert np.abs(Fs - F).max() < 1e-13
    assert np.abs(Zs.sum(0) - Z).max() < 1e-13


# ----------------------------------------------------------------------------
# brute force on tiny inputs
# ----------------------------------------------------------------------------

def _tiny(seed=2, grid=(6, 7, 9)):
    rng = np.random.default_rng(seed)
    sp1 = I.make_species("X", "spd", 3.2, 0.01, rng)
    sp2 = I.make_species("Y", "sp", 2.7, 0.01, rng)
    cell = np.array([[3.9, 0.0, 0.0], [0.8, 4.2, 0.0], [0.2, 0.5, 3.6]])
    pos = np.array([[0.3, 0.2, 0.1], [2.1, 2.4, 1.9], [1.0, 3.7, 2.8]])
    millers = I.random_millers_box(rng, 5, 2)
    v = I.plane_wave_potential(grid, millers, np.full(5, 0.4), rng.uniform(0, 6.28, 5))
    return I.assemble(cell, pos, np.array([0, 1, 0]), [sp1, sp2], grid, v, rng)


def test_brute_force_tiny(oracle_mod):
    """Triple loop over (point, atom, image box) with its own enumeration, and
    the Gamma-point dense product Phi^T diag(wV) Phi, agree with the oracle
    (H, rho, and the magnitude scale sum |phi||D||phi| of rho's terms)."""
    s = _tiny()
    o = oracle_mod.Oracle(s)
    N = s.grid
    w = s.volume / s.ngrid
    norb = s.norb_atom()
    rc = s.rcut_atom()
    idx = I.block_index(s.blk_i, s.blk_j, s.blk_r)
    Ts = np.array(np.meshgrid(*[np.arange(-4, 5)] * 3, indexing="ij")).reshape(3, -1).T
    H = np.zeros(s.nnz)
    rho = np.zeros(s.ngrid)
    rho_abs = np.zeros(s.ngrid)
    ostart = np.concatenate([[0], np.cumsum(norb)])
    Phi = np.zeros((s.ngrid, int(ostart[-1])))
    W = 0.0
    for g in range(s.ngrid):
        n = np.array([g // (N[1] * N[2]), (g // N[2]) % N[1], g % N[2]])
        r = (n / N) @ s.cell
        ent = []
        for a in range(s.natom):
            x = r - s.pos[a] - Ts @ s.cell
            ok = np.linalg.norm(x, axis=1) < rc[a]
            for T, xx in zip(Ts[ok], x[ok]):
                phi, _ = o.orbitals(int(s.species[a]), xx)
                ent.append((a, T, phi[0]))
                Phi[g, ostart[a]:ostart[a + 1]] += phi[0]
        # unit of work: ordered orbital pairs of the point's neighbour images
        W += float(sum(norb[a] for (a, _, _) in ent)) ** 2
        for (a, T, pa) in ent:
            for (b, T2, pb) in ent:
                R = T2 - T
                k = idx[(a, b, int(R[0]), int(R[1]), int(R[2]))]
                blk = np.outer(pa, pb)
                H[s.blk_off[k]:s.blk_off[k] + blk.size] += w * s.v[g] * blk.ravel()
                D = s.d[s.blk_off[k]:s.blk_off[k] + blk.size].reshape(blk.shape)
                rho[g] += np.sum(D * blk)
                rho_abs[g] += np.sum(np.abs(D) * np.abs(blk))
    Ho = o.vlocal()
    assert np.abs(Ho - H).max() < 1e-14 * max(1, np.abs(H).max()) * 10
    # W = sum_g n_orb(g)^2: integers, so exact
    assert o.work() == W
    assert np.abs(o.rho() - rho).max() < 1e-13 * max(1, np.abs(rho).max())
    # magnitude scale of rho's terms (the bound of the reduced-precision tests)
    ra = o.rho_abs()
    assert np.abs(ra - rho_abs).max() < 1e-13 * rho_abs.max()
    assert np.all(ra >= np.abs(rho) * (1 - 1e-14))
    # dense Gamma-point check: the oracle's fold of H(I,J,R) over R equals
    # Phi^T diag(wV) Phi with Phi the orbitals summed over lattice images
    HG = Phi.T @ (Phi * (w * s.v)[:, None])
    HGo = o.fold_gamma(Ho)
    assert np.abs(HG - HGo).max() < 1e-13 * np.abs(HG).max()
    SG = Phi.T @ (Phi * w)
    assert np.abs(SG - o.fold_gamma(o.vlocal(np.ones(s.ngrid)))).max() < 1e-13 * np.abs(SG).max()


# ----------------------------------------------------------------------------
# invariances
# ----------------------------------------------------------------------------

def test_grid_translation_invariance(oracle_mod):
    s = I.diamond8(1, grid=(16, 16, 16))
    o = oracle_mod.Oracle(s)
    h0, rho0 = o.vlocal(), o.rho()
    F0, Z0, E0, _ = o.force_stress()
    shift = np.array([2, 1, 3])
    s2 = I.diamond8(1, grid=(16, 16, 16))
    s2.pos = s.pos + (shift / s.grid) @ s.cell
    v3 = s.v.reshape(tuple(s.grid))
    s2.v = np.roll(v3, tuple(shift), axis=(0, 1, 2)).ravel().copy()
    o2 = oracle_mod.Oracle(s2)
    h2, rho2 = o2.vlocal(), o2.rho()
    F2, Z2, E2, _ = o2.force_stress()
    assert np.abs(h2 - h0).max() < 1e-12
    assert np.abs(rho2.reshape(v3.shape) - np.roll(rho0.reshape(v3.shape), tuple(shift), axis=(0, 1, 2))).max() < 1e-12
    assert np.abs(F2 - F0).max() < 1e-11 and np.abs(Z2 - Z0).max() < 1e-11


def test_atom_permutation(oracle_mod):
    s = _tiny(3, grid=(8, 8, 8))
    o = oracle_mod.Oracle(s)
    h, F = o.vlocal(), o.force_stress()[0]
    perm = np.array([2, 0, 1])          # new atom k is old atom perm[k]
    inv = np.argsort(perm)
    rng = np.random.default_rng(0)
    s2 = I.assemble(s.cell, s.pos[perm], s.species[perm], s.species_list, s.grid, s.v, rng)
    # carry D over block by block
    idx1 = I.block_index(s.blk_i, s.blk_j, s.blk_r)
    d2 = np.zeros(s2.nnz)
    for k in range(len(s2.blk_i)):
        a, b, r = perm[s2.blk_i[k]], perm[s2.blk_j[k]], s2.blk_r[k]
        k1 = idx1[(int(a), int(b), int(r[0]), int(r[1]), int(r[2]))]
        n = s.norb_atom()[a] * s.norb_atom()[b]
        d2[s2.blk_off[k]:s2.blk_off[k] + n] = s.d[s.blk_off[k1]:s.blk_off[k1] + n]
    s2.d = d2
    o2 = oracle_mod.Oracle(s2)
    h2, F2 = o2.vlocal(), o2.force_stress()[0]
    for k in range(len(s2.blk_i)):
        a, b, r = perm[s2.blk_i[k]], perm[s2.blk_j[k]], s2.blk_r[k]
        k1 = idx1[(int(a), int(b), int(r[0]), int(r[1]), int(r[2]))]
        n = s.norb_atom()[a] * s.norb_atom()[b]
        assert np.abs(h2[s2.blk_off[k]:s2.blk_off[k] + n] - h[s.blk_off[k1]:s.blk_off[k1] + n]).max() < 1e-14
    assert np.abs(F2 - F[perm]).max() < 1e-12


def test_linearity(oracle_mod):
    s = _tiny(4, grid=(8, 8, 8))
    o = oracle_mod.Oracle(s)
    rng = np.random.default_rng(1)
    v1, v2 = rng.normal(size=s.ngrid), rng.normal(size=s.ngrid)
    h = o.vlocal(v=2 * v1 - 3 * v2)
    assert np.abs(h - (2 * o.vlocal(v=v1) - 3 * o.vlocal(v=v2))).max() < 1e-13
    d1 = s.d
    r = o.rho(d=2.5 * d1)
    assert np.abs(r - 2.5 * o.rho()).max() < 1e-13
    F1 = o.force_stress(v=v1)[0]
    F2 = o.force_stress(v=v2)[0]
    assert np.abs(o.force_stress(v=v1 + v2)[0] - (F1 + F2)).max() < 1e-12


# ----------------------------------------------------------------------------
# finite differences (table mode with the smooth cutoff)
# ----------------------------------------------------------------------------

def _energy(oracle_mod, s):
    return oracle_mod.Oracle(s).force_stress()[2]


def test_force_finite_difference(oracle_mod):
    s = I.diamond8(0, grid=(24, 24, 24))
    F, Z, E, _ = oracle_mod.Oracle(s).force_stress()
    dR = 1e-4
    for K in (0, 5):
        for a in range(3):
            sp, sm = I.diamond8(0, grid=(24, 24, 24)), I.diamond8(0, grid=(24, 24, 24))
            sp.pos = s.pos.copy(); sp.pos[K, a] += dR
            sm.pos = s.pos.copy(); sm.pos[K, a] -= dR
            fd = -(_energy(oracle_mod, sp) - _energy(oracle_mod, sm)) / (2 * dR)
            assert abs(fd - F[K, a]) < 2e-6 * np.abs(F).max(), (K, a, fd, F[K, a])


def test_strain_finite_difference(oracle_mod):
    s = I.diamond8(0, grid=(24, 24, 24))
    F, Z, E, _ = oracle_mod.Oracle(s).force_stress()
    de = 1e-5
    for a in range(3):
        for b in range(3):
            vals = []
            for sgn in (1, -1):
                M = np.eye(3)
                M[a, b] += sgn * de
                st = I.diamond8(0, grid=(24, 24, 24))
                st.pos = s.pos @ M.T
                st.cell = s.cell @ M.T
                vals.append(_energy(oracle_mod, st) / np.linalg.det(M))   # w held fixed
            fd = (vals[0] - vals[1]) / (2 * de)
            assert abs(fd - Z[a, b]) < 2e-6 * np.abs(Z).max(), (a, b, fd, Z[a, b])


# ----------------------------------------------------------------------------
# orbitals
# ----------------------------------------------------------------------------

def _orb_system(oracle_mod, cutoff=False, dr=0.01, alphas=(1.0, 1.0, 1.0), rc=8.0):
    rng = np.random.default_rng(0)
    sp = I.make_species("Q", "spd", rc, dr, rng, alphas=list(alphas), cutoff=cutoff)
    s = I.assemble(np.eye(3) * 20, np.zeros((1, 3)), np.array([0]), [sp], (4, 4, 4), np.zeros(64), rng)
    return s, sp


def test_ylm_orthonormal_and_addition_theorem(oracle_mod):
    s, sp = _orb_system(oracle_mod)
    o = oracle_mod.Oracle(s, radial="analytic")
    xg, wg = np.polynomial.legendre.leggauss(10)
    nphi = 20
    ph = 2 * np.pi * np.arange(nphi) / nphi
    ct, pp = np.meshgrid(xg, ph, indexing="ij")
    st = np.sqrt(1 - ct**2)
    u = np.stack([st * np.cos(pp), st * np.sin(pp), ct], -1).reshape(-1, 3)
    wq = (np.outer(wg, np.full(nphi, 2 * np.pi / nphi))).ravel()
    phi, _ = o.orbitals(0, u)           # r = 1: phi = exp(-1) Y_lm
    Y = phi / math.exp(-1.0)
    G = Y.T @ (Y * wq[:, None])
    assert np.abs(G - np.eye(9)).max() < 1e-13
    # sum_m Y_lm^2 = (2l+1)/(4 pi)
    for l, sl in ((0, slice(0, 1)), (1, slice(1, 4)), (2, slice(4, 9))):
        assert np.abs((Y[:, sl] ** 2).sum(1) - (2 * l + 1) / (4 * math.pi)).max() < 1e-13


def test_ylm_m_convention(oracle_mod):
    """m < 0 are sin-type (odd under y -> -y), m >= 0 even; rotating about z by
    t turns the (m, -m) pair by |m| t and leaves m = 0 fixed."""
    s, sp = _orb_system(oracle_mod)
    o = oracle_mod.Oracle(s, radial="analytic")
    rng = np.random.default_rng(3)
    x = rng.normal(size=(20, 3))
    x /= np.linalg.norm(x, axis=1)[:, None]
    y = x * np.array([1, -1, 1])
    p1, _ = o.orbitals(0, x)
    p2, _ = o.orbitals(0, y)
    ms = [0, -1, 0, 1, -2, -1, 0, 1, 2]
    for k, m in enumerate(ms):
        sgn = -1 if m < 0 else 1
        assert np.abs(p2[:, k] - sgn * p1[:, k]).max() < 1e-14
    t = 0.37
    R = np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0], [0, 0, 1]])
    pr, _ = o.orbitals(0, x @ R.T)
    for (kneg, kpos, m) in ((1, 3, 1), (5, 7, 1), (4, 8, 2)):
        c, s_ = math.cos(m * t), math.sin(m * t)
        # f(R^-1 x) rotates cos/sin pairs: Y_c(Rx) = c Y_c - s Y_s, Y_s(Rx) = s Y_c + c Y_s
        assert np.abs(pr[:, kpos] - (c * p1[:, kpos] - s_ * p1[:, kneg])).max() < 1e-13
        assert np.abs(pr[:, kneg] - (s_ * p1[:, kpos] + c * p1[:, kneg])).max() < 1e-13
    for k in (0, 2, 6):
        assert np.abs(pr[:, k] - p1[:, k]).max() < 1e-13


@pytest.mark.parametrize("radial", ["analytic", "table"])
def test_orbital_gradient_fd(oracle_mod, radial):
    s, sp = _orb_system(oracle_mod, cutoff=True, alphas=(0.8, 1.3, 0.5), rc=6.0)
    o = oracle_mod.Oracle(s, radial=radial)
    rng = np.random.default_rng(4)
    x = rng.uniform(-3.5, 3.5, size=(40, 3))
    x = x[np.linalg.norm(x, axis=1) < 5.9]
    phi, grad = o.orbitals(0, x)
    hstep = 1e-6
    for a in range(3):
        e = np.zeros(3); e[a] = hstep
        fd = (o.orbitals(0, x + e)[0] - o.orbitals(0, x - e)[0]) / (2 * hstep)
        assert np.abs(fd - grad[:, :, a]).max() < 1e-8


def test_hermite_interpolant_bound(oracle_mod):
    """Knot values are exact; between knots |p - f| <= dr^4 max|f''''|/384 and
    |p' - f'| <= (sqrt3/216) dr^3 max|f''''| for f = exp(-a r^2)."""
    dr = 0.01
    s, sp = _orb_system(oracle_mod, cutoff=False, dr=dr, alphas=(2.0, 1.0, 0.5), rc=7.0)
    ot = oracle_mod.Oracle(s, radial="table")
    oa = oracle_mod.Oracle(s, radial="analytic")
    rk = np.arange(0, 690) * dr
    p, dp = ot.radial(0, 0, rk)
    assert np.abs(p - sp.f[0][:690]).max() < 1e-15
    assert np.abs(dp - sp.fp[0][:690]).max() < 1e-14
    r = np.random.default_rng(9).uniform(0, 6.9, 20000)
    for c, a in enumerate(sp.alphas):
        pt, dpt = ot.radial(0, c, r)
        pa, dpa = oa.radial(0, c, r)
        f4 = 12 * a * a           # max |d^4/dr^4 exp(-a r^2)| is at r = 0
        assert np.abs(pt - pa).max() <= dr**4 * f4 / 384 * 1.0001
        assert np.abs(dpt - dpa).max() <= math.sqrt(3) / 216 * dr**3 * f4 * 1.0001


def test_radial_cutoff_edge(oracle_mod):
    """r within one ulp of rcut stays inside the table (index clamped) and the
    tapered function vanishes there; r >= rcut gives exactly zero."""
    s, sp = _orb_system(oracle_mod, cutoff=True, alphas=(0.3, 0.3, 0.3), rc=6.0)
    o = oracle_mod.Oracle(s, radial="table")
    r = np.array([np.nextafter(6.0, 0.0), 6.0, 6.5])
    p, dp = o.radial(0, 2, r)
    assert abs(p[0]) < 1e-15 and p[1] == 0.0 and p[2] == 0.0


# ----------------------------------------------------------------------------
# unit of work W = sum_g n_orb(g)^2 and the smooth cutoff
# ----------------------------------------------------------------------------

def test_work_units_enumeration(oracle_mod):
    """W counted by the oracle's cell lists equals a vectorised enumeration of
    every (point, atom, image) within rcut over a box of images wider than the
    cutoff, on the jittered diamond (rcut 6 > cell edge 6.74 / 2) and on a
    sub-range of grid points."""
    s = I.diamond8(0, grid=(12, 14, 10))
    o = oracle_mod.Oracle(s)
    N = np.asarray(s.grid)
    n = np.stack(np.meshgrid(*[np.arange(k) for k in N], indexing="ij"), -1).reshape(-1, 3)
    r = (n / N) @ s.cell
    Ts = np.array(np.meshgrid(*[np.arange(-3, 4)] * 3, indexing="ij")).reshape(3, -1).T
    shifts = Ts @ s.cell
    rc, norb = s.rcut_atom(), s.norb_atom()
    count = np.zeros(len(r))
    for a in range(s.natom):
        x = r[:, None, :] - s.pos[a][None, None, :] - shifts[None, :, :]
        inside = np.sqrt((x * x).sum(-1)) < rc[a]
        # the box of images is wide enough: no image on its faces is in range
        edge = np.abs(Ts).max(1) == 3
        assert not inside[:, edge].any()
        count += norb[a] * inside.sum(1)
    assert o.work() == float((count ** 2).sum())
    g0, g1 = 317, 1201
    assert o.work(g_range=(g0, g1)) == float((count[g0:g1] ** 2).sum())


def _taper_species(oracle_mod, rs_frac=0.75, rc=6.0, alphas=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(1)
    sp = I.make_species("T", "spd", rc, 0.01, rng, alphas=list(alphas), rs_frac=rs_frac, cutoff=True)
    s = I.assemble(np.eye(3) * 20, np.zeros((1, 3)), np.array([0]), [sp], (4, 4, 4), np.zeros(64), rng)
    return s, sp


def test_taper_is_the_c2_quintic_step(oracle_mod):
    """With a = 0 the analytic radial function is the taper chi alone.  The
    smooth cutoff is C2: chi = 1 up to r_s and 0 from rcut, with chi, chi' and
    chi'' continuous at both ends.  A polynomial of degree <= 5 in
    t = (r - r_s)/(rcut - r_s) is fixed uniquely by those six end conditions,
    so checking degree <= 5 (a degree-5 fit leaves no residual), the values
    and first derivatives (the oracle's own chi') and the second derivatives
    (finite differences of chi') at both ends pins chi without restating it.
    The step is also point-symmetric: chi(r_s + u) + chi(rcut - u) = 1."""
    rc, rs = 6.0, 4.5
    s, sp = _taper_species(oracle_mod)
    o = oracle_mod.Oracle(s, radial="analytic")
    inner = np.linspace(0.0, rs, 31)
    p, dp = o.radial(0, 0, inner)
    assert np.all(p == 1.0) and np.all(dp == 0.0)
    outer = np.array([rc, rc + 1e-9, 7.0])
    p, dp = o.radial(0, 0, outer)
    assert np.all(p == 0.0) and np.all(dp == 0.0)
    # degree <= 5 on (r_s, rcut)
    t = np.linspace(0.02, 0.98, 41)
    p, dp = o.radial(0, 0, rs + t * (rc - rs))
    coef = np.polynomial.polynomial.polyfit(t, p, 5)
    assert np.abs(np.polynomial.polynomial.polyval(t, coef) - p).max() < 1e-14
    # end conditions from the fitted polynomial (exact up to the fit's
    # conditioning): it meets chi = 1 at t = 0 and chi = 0 at t = 1 with zero
    # slope and curvature on both sides
    P = np.polynomial.Polynomial(coef)
    for t0, val in ((0.0, 1.0), (1.0, 0.0)):
        assert abs(P(t0) - val) < 1e-11
        assert abs(P.deriv(1)(t0)) < 1e-9
        assert abs(P.deriv(2)(t0)) < 1e-7
    # the oracle's chi' is the derivative of that polynomial
    assert np.abs(dp * (rc - rs) - P.deriv(1)(t)).max() < 1e-9
    # point symmetry about the midpoint, and chi(mid) = 1/2
    u = np.linspace(0.0, rc - rs, 17)
    pa, _ = o.radial(0, 0, rs + u)
    pb, _ = o.radial(0, 0, rc - u)
    assert np.abs(pa + pb - 1.0).max() < 1e-15 * 8
    pm, _ = o.radial(0, 0, np.array([0.5 * (rs + rc)]))
    assert abs(pm[0] - 0.5) < 1e-15
    # the six end conditions leave exactly one quintic; its slope at the midpoint
    # is -15/8 per unit t (the derivative of the unique C2 step)
    _, dmid = o.radial(0, 0, np.array([0.5 * (rs + rc)]))
    assert abs(dmid[0] * (rc - rs) + 15.0 / 8.0) < 1e-13


def test_taper_tables_match_analytic(oracle_mod):
    """With the cutoff on, the tabulated radial functions (built by the input
    generator) interpolated by the oracle's table mode agree with the oracle's
    own analytic f = exp(-a r^2) chi(r) within the cubic Hermite error bound
    dr^4 max|f''''| / 384 (max|f''''| from finite differences of the
    analytic f), over the whole range including the taper region."""
    s, sp = _taper_species(oracle_mod, alphas=(0.35, 1.1, 1.9))
    ot = oracle_mod.Oracle(s, radial="table")
    oa = oracle_mod.Oracle(s, radial="analytic")
    rng = np.random.default_rng(5)
    r = np.concatenate([rng.uniform(0.0, 6.0, 20000), rng.uniform(4.4, 6.0, 20000)])
    hf = 2e-3
    rf = np.arange(0.0, 6.0 + hf, hf)
    for c in range(3):
        pt, _ = ot.radial(0, c, r)
        pa, _ = oa.radial(0, c, r)
        fa, _ = oa.radial(0, c, rf)
        # fourth differences of an even function: extend to r < 0 by symmetry
        ext = np.concatenate([fa[:0:-1], fa])
        d4 = np.abs(np.diff(ext, 4)).max() / hf**4
        bound = 0.01**4 * d4 / 384
        err = np.abs(pt - pa).max()
        assert err <= 1.2 * bound, (c, err, bound)
        assert err > 0.0     # the table is an interpolant, not the function


# ----------------------------------------------------------------------------
# one SCF step at the Gamma point
# ----------------------------------------------------------------------------

def test_gamma_fold_scatter_duality(oracle_mod):
    """scatter_gamma is the adjoint of fold_gamma over the pattern:
    <scatter(M), X>_blocks = <M, fold(X)>_dense for any M and X (an
    off-by-one block offset or a transposed tile breaks it)."""
    s = _tiny()
    o = oracle_mod.Oracle(s)
    rng = np.random.default_rng(3)
    n = int(s.norb_atom().sum())
    M = rng.standard_normal((n, n))
    X = rng.standard_normal(s.nnz)
    assert abs(np.dot(o.scatter_gamma(M), X) - np.sum(M * o.fold_gamma(X))) < 1e-12 * np.abs(X).sum()


@pytest.mark.parametrize("kT", [0.0, 0.05])
def test_scf_gamma_step(oracle_mod, kT):
    """The reference SCF step solves H c = e S c (residual and S-orthonormality
    of the eigenvectors), fills n_electrons, and its D(R) puts exactly that
    many electrons on the grid: N_e = sum_g w rho_g = <D, S>_blocks = sum f."""
    from paper_2409_09399_amd import inputs as I
    s = I.diamond8(0, grid=(12, 12, 12))
    o = oracle_mod.Oracle(s)
    h = o.vlocal()
    sv = o.vlocal(np.ones(s.ngrid))
    nel = 32.0 if kT == 0 else 31.0
    e, f, Z, D = o.scf_gamma(h, sv, nel, kT)
    HG, SG = o.fold_gamma(h), o.fold_gamma(sv)
    assert np.all(np.diff(e) >= 0)
    assert np.abs(HG @ Z - (SG @ Z) * e).max() < 1e-9 * np.abs(e).max()
    assert np.abs(Z.T @ SG @ Z - np.eye(len(e))).max() < 1e-9
    assert abs(f.sum() - nel) < 1e-10
    assert np.all((f >= 0) & (f <= 2))
    if kT == 0:
        assert np.array_equal(f[:16], np.full(16, 2.0)) and not f[16:].any()
    w = s.volume / s.ngrid
    assert abs(float(np.dot(D, sv)) - nel) < 1e-9 * nel
    assert abs(o.rho(D).sum() * w - nel) < 1e-9 * nel

