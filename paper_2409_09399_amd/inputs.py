"""Seeded synthetic inputs for grid integration ("Gint").

This module only *builds inputs*: geometries, species radial tables, the
block pattern of the sparse density matrix, a local potential on the grid and
random density-matrix values.  It holds none of the grid-integration
arithmetic (no orbital products, no sums over the grid), so both the HIP path
and the FP64 CPU oracle can consume what it produces without sharing any code
with each other.

Workloads follow the paper's benchmark family: twisted bilayer graphene
(Results, "Testing Systems" and Table 2) built as commensurate cells, plus a
small jittered diamond cell for exact parity work.  Units: Bohr and Hartree.

Radial functions (the inputs of the orbital definition phi = R_l(r) Y_lm):
R_c(r) = r^l f_c(r), f_c(r) = exp(-a_c r^2) chi(r) with the C2 smooth cutoff
chi(r) = 1 for r <= r_s, 1 - (10 t^3 - 15 t^4 + 6 t^5) with
t = (r - r_s)/(rcut - r_s) for r_s < r < rcut, 0 beyond.  The tables store
f and f' at knots r_k = k dr, k = 0..ceil(rcut/dr).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BOHR_PER_ANGSTROM = 1.8897259886

# Channel angular momenta per basis label; orbitals are ordered by channel
# (l ascending, then zeta), then m = -l..l.
BASIS_CHANNELS = {
    "2s2p1d": (0, 0, 1, 1, 2),   # 13 orbitals (C, O)
    "2s1p": (0, 0, 1),           # 5 orbitals (H)
    "sp": (0, 1),                # 4 orbitals (closed-form tests)
    "spd": (0, 1, 2),            # 9 orbitals (one channel per l)
}


@dataclasses.dataclass
class Species:
    name: str
    rcut: float
    dr: float
    ls: np.ndarray          # int32 [nchan]
    alphas: np.ndarray      # float64 [nchan] Gaussian exponents (analytic form)
    f: np.ndarray           # float64 [nchan, nknots] table of f(r_k)
    fp: np.ndarray          # float64 [nchan, nknots] table of f'(r_k)
    rs: float               # start of the smooth cutoff; rcut == rs means no taper
    cutoff: bool = True     # False: plain Gaussian, no taper (closed-form tests)

    @property
    def nknots(self) -> int:
        return int(self.f.shape[1])

    @property
    def nchan(self) -> int:
        return int(self.ls.shape[0])

    @property
    def norb(self) -> int:
        return int(sum(2 * int(l) + 1 for l in self.ls))


@dataclasses.dataclass
class System:
    cell: np.ndarray        # float64 [3,3], rows are lattice vectors a1,a2,a3
    pos: np.ndarray         # float64 [natom,3] Cartesian, used as given
    species: np.ndarray     # int32 [natom]
    species_list: List[Species]
    grid: np.ndarray        # int32 [3]
    blk_i: np.ndarray       # int32 [nblk]
    blk_j: np.ndarray       # int32 [nblk]
    blk_r: np.ndarray       # int32 [nblk,3]
    blk_off: np.ndarray     # int64 [nblk]
    nnz: int
    v: np.ndarray           # float64 [N1*N2*N3] local potential, C order
    d: np.ndarray           # float64 [nnz] density matrix over the pattern
    name: str = ""

    @property
    def natom(self) -> int:
        return int(self.pos.shape[0])

    @property
    def ngrid(self) -> int:
        return int(np.prod(self.grid))

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.cell)))

    def norb_atom(self) -> np.ndarray:
        return np.array([self.species_list[s].norb for s in self.species], dtype=np.int64)

    def rcut_atom(self) -> np.ndarray:
        return np.array([self.species_list[s].rcut for s in self.species], dtype=np.float64)


# ----------------------------------------------------------------------------
# Radial tables
# ----------------------------------------------------------------------------

def _taper(r: np.ndarray, rs: float, rc: float):
    """Smooth cutoff chi(r) and chi'(r) (C2 quintic taper between rs and rc)."""
    chi = np.ones_like(r)
    dchi = np.zeros_like(r)
    if rc > rs:
        t = (r - rs) / (rc - rs)
        mid = (r > rs) & (r < rc)
        tm = t[mid]
        chi[mid] = 1.0 - (10 * tm**3 - 15 * tm**4 + 6 * tm**5)
        dchi[mid] = -(30 * tm**2 - 60 * tm**3 + 30 * tm**4) / (rc - rs)
    chi[r >= rc] = 0.0
    dchi[r >= rc] = 0.0
    return chi, dchi


def make_species(name: str, basis, rcut: float, dr: float,
                 rng: np.random.Generator, alpha_range=(0.3, 2.0),
                 rs_frac: float = 0.75, alphas: Optional[Sequence[float]] = None,
                 cutoff: bool = True) -> Species:
    ls = np.array(BASIS_CHANNELS[basis] if isinstance(basis, str) else basis, dtype=np.int32)
    if alphas is None:
        alphas = rng.uniform(alpha_range[0], alpha_range[1], size=ls.shape[0])
    alphas = np.asarray(alphas, dtype=np.float64)
    nk = int(math.ceil(rcut / dr - 1e-12)) + 1
    r = np.arange(nk, dtype=np.float64) * dr
    rs = rs_frac * rcut if cutoff else rcut
    if cutoff:
        chi, dchi = _taper(r, rs, rcut)
    else:
        chi, dchi = np.ones_like(r), np.zeros_like(r)
    f = np.empty((ls.shape[0], nk))
    fp = np.empty((ls.shape[0], nk))
    for c, a in enumerate(alphas):
        g = np.exp(-a * r * r)
        f[c] = g * chi
        fp[c] = -2.0 * a * r * g * chi + g * dchi
    return Species(name=name, rcut=float(rcut), dr=float(dr), ls=ls, alphas=alphas,
                   f=f, fp=fp, rs=float(rs), cutoff=cutoff)


# ----------------------------------------------------------------------------
# Geometry
# ----------------------------------------------------------------------------

def diamond_cell(a: float = 6.74, jitter_sigma: float = 0.05, rng=None):
    """8 atoms at the diamond sites of a cubic cell, plus a uniform jitter of
    standard deviation jitter_sigma on each Cartesian component."""
    frac = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                     [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])
    cell = np.eye(3) * a
    pos = frac @ cell
    if rng is not None and jitter_sigma > 0:
        half = math.sqrt(3.0) * jitter_sigma
        pos = pos + rng.uniform(-half, half, size=pos.shape)
    return cell, pos


def tbg_twist_angle(i: int) -> float:
    """Commensurate twist angle (radians) of the (i, i+1) bilayer cell."""
    q = 3 * i * i + 3 * i + 1
    return math.acos((q - 0.5) / q)


def tbg_atom_count(i: int) -> int:
    return 4 * (3 * i * i + 3 * i + 1)


def tbg(i: int, a_ang: float = 2.46, d_ang: float = 3.35, vacuum: float = 20.0):
    """Commensurate twisted bilayer graphene (standard construction).

    Layer 1: graphene with a1 = a(1,0), a2 = a(1/2, sqrt3/2) and basis 0 and
    (a1+a2)/3 at z = 0.  The superlattice is t1 = i a1 + (i+1) a2,
    t2 = -(i+1) a1 + (2i+1) a2 (60 degrees apart).  Layer 2 is layer 1
    rotated by the commensurate angle (which maps (i+1) a1 + i a2 onto t1)
    and lifted by d.  The third cell vector is (0, 0, d + vacuum).
    Returns (cell [3,3] Bohr, pos [N,3] Bohr, theta radians)."""
    a = a_ang * BOHR_PER_ANGSTROM
    d = d_ang * BOHR_PER_ANGSTROM
    a1 = np.array([a, 0.0])
    a2 = np.array([0.5 * a, 0.5 * math.sqrt(3.0) * a])
    t1 = i * a1 + (i + 1) * a2
    t2 = -(i + 1) * a1 + (2 * i + 1) * a2
    theta = tbg_twist_angle(i)
    c, s = math.cos(theta), math.sin(theta)
    rot = np.array([[c, -s], [s, c]])
    tinv = np.linalg.inv(np.stack([t1, t2]))   # frac = xy @ tinv
    per_layer = 2 * (3 * i * i + 3 * i + 1)
    layers = []
    for layer in range(2):
        b1, b2 = (a1, a2) if layer == 0 else (rot @ a1, rot @ a2)
        basis = [np.zeros(2), (b1 + b2) / 3.0]
        nmax = 3 * (i + 2)
        n1, n2 = np.meshgrid(np.arange(-nmax, nmax + 1), np.arange(-nmax, nmax + 1), indexing="ij")
        lat = n1.reshape(-1, 1) * b1 + n2.reshape(-1, 1) * b2
        pts = []
        for bvec in basis:
            xy = lat + bvec
            fr = xy @ tinv
            fr = fr - np.floor(fr + 1e-9)
            fr[np.abs(fr - 1.0) < 1e-9] = 0.0
            pts.append(fr)
        fr = np.concatenate(pts)
        key = np.round(fr * 1e6).astype(np.int64)
        _, idx = np.unique(key, axis=0, return_index=True)
        fr = fr[np.sort(idx)]
        if fr.shape[0] != per_layer:
            raise RuntimeError(f"TBG layer {layer}: {fr.shape[0]} sites, expected {per_layer}")
        xy = fr @ np.stack([t1, t2])
        z = np.full((xy.shape[0], 1), layer * d)
        layers.append(np.hstack([xy, z]))
    pos = np.concatenate(layers)
    cell = np.array([[t1[0], t1[1], 0.0], [t2[0], t2[1], 0.0], [0.0, 0.0, d + vacuum]])
    return cell, pos, theta


def grid_for_spacing(cell: np.ndarray, h: float, multiple: int = 8) -> np.ndarray:
    lens = np.linalg.norm(cell, axis=1)
    n = np.maximum(1, np.round(lens / (h * multiple))).astype(np.int64) * multiple
    return n.astype(np.int32)


# ----------------------------------------------------------------------------
# Block pattern, local potential, density matrix
# ----------------------------------------------------------------------------

def _image_range(cell: np.ndarray, reach: float) -> np.ndarray:
    """Integer bounds n_i such that every lattice vector T with |T h| <= reach
    has |T_i| <= n_i (interplanar spacings of the cell)."""
    recip = np.linalg.inv(cell).T            # rows b_i with a_i . b_j = delta_ij
    spacing = 1.0 / np.linalg.norm(recip, axis=1)
    return np.ceil(reach / spacing).astype(np.int64) + 1


def build_pattern(cell, pos, rcut_atom, skin: float = 0.5):
    """All (I, J, R) with |tau_J + R h - tau_I| < rc_I + rc_J + skin.
    Returns int32 I, J, int32 R[nblk,3] in (I, J, R) lexicographic order."""
    from scipy.spatial import cKDTree
    natom = pos.shape[0]
    rmax = float(np.max(rcut_atom))
    reach = 2.0 * rmax + skin
    span = float(np.max(np.linalg.norm(pos - pos.mean(0), axis=1)))
    nr = _image_range(cell, reach + 2.0 * span)
    rr = np.stack(np.meshgrid(*[np.arange(-n, n + 1) for n in nr], indexing="ij"), -1).reshape(-1, 3)
    shifts = rr @ cell
    img = (pos[None, :, :] + shifts[:, None, :]).reshape(-1, 3)
    pairs = cKDTree(pos).query_ball_tree(cKDTree(img), reach)
    cnt = np.fromiter((len(h) for h in pairs), dtype=np.int64, count=natom)
    i = np.repeat(np.arange(natom, dtype=np.int64), cnt)
    h = np.fromiter((x for hh in pairs for x in hh), dtype=np.int64, count=int(cnt.sum()))
    j = h % natom
    r = rr[h // natom]
    dist = np.linalg.norm(img[h] - pos[i], axis=1)
    keep = dist < rcut_atom[i] + rcut_atom[j] + skin
    bi = i[keep].astype(np.int32)
    bj = j[keep].astype(np.int32)
    br = r[keep].astype(np.int32)
    order = np.lexsort((br[:, 2], br[:, 1], br[:, 0], bj, bi))
    return bi[order], bj[order], br[order]


def block_offsets(bi, bj, norb_atom) -> np.ndarray:
    sizes = norb_atom[bi] * norb_atom[bj]
    off = np.zeros(bi.shape[0], dtype=np.int64)
    if bi.shape[0] > 1:
        off[1:] = np.cumsum(sizes[:-1])
    return off


def _canonical(bi, bj, br) -> np.ndarray:
    """True for blocks on the canonical half: I < J, or I == J and R >= 0
    lexicographically."""
    rpos = (br[:, 0] > 0) | ((br[:, 0] == 0) & ((br[:, 1] > 0) | ((br[:, 1] == 0) & (br[:, 2] >= 0))))
    return (bi < bj) | ((bi == bj) & rpos)


def block_index(bi, bj, br) -> dict:
    return {(int(i), int(j), int(r[0]), int(r[1]), int(r[2])): k
            for k, (i, j, r) in enumerate(zip(bi, bj, br))}


def _block_keys(bi, bj, br, natom: int, m: int) -> np.ndarray:
    """int64 keys that sort like (I, J, R) lexicographically, for |R_i| <= m."""
    base = 2 * m + 1
    if float(natom) ** 2 * float(base) ** 3 >= 2.0 ** 62:
        raise ValueError("pattern too large for int64 block keys")
    k = bi.astype(np.int64) * natom + bj.astype(np.int64)
    for c in range(3):
        k = k * base + (br[:, c].astype(np.int64) + m)
    return k


def transpose_index(bi, bj, br, natom: int) -> np.ndarray:
    """For each block (I, J, R) the index of (J, I, -R); -1 if absent.
    Blocks must be in (I, J, R) lexicographic order."""
    m = int(np.abs(br).max()) if br.size else 0
    keys = _block_keys(bi, bj, br, natom, m)
    kt = _block_keys(bj, bi, -br, natom, m)
    pos = np.searchsorted(keys, kt)
    pos = np.minimum(pos, keys.shape[0] - 1)
    return np.where(keys[pos] == kt, pos, -1)


def random_density_matrix(cell, pos, bi, bj, br, off, norb_atom, rng, decay=3.0):
    """D_IJR[mu,nu] = u exp(-|d_IJR|/decay), u ~ U[-1/2, 1/2], drawn on the
    canonical half (block by block in pattern order, each row-major) and
    transposed into the other half; the (I,I,0) blocks are symmetrised and
    get +1 on the diagonal.  Satisfies D_JI(-R) = D_IJR^T."""
    natom = pos.shape[0]
    nnz = int(off[-1] + norb_atom[bi[-1]] * norb_atom[bj[-1]])
    d = np.zeros(nnz)
    tr = transpose_index(bi, bj, br, natom)
    if np.any(tr < 0):
        raise ValueError("pattern is not transpose-closed")
    ks = np.nonzero(_canonical(bi, bj, br))[0]
    ni = norb_atom[bi[ks]].astype(np.int64)
    nj = norb_atom[bj[ks]].astype(np.int64)
    size = ni * nj
    ustart = np.zeros(ks.shape[0], dtype=np.int64)
    ustart[1:] = np.cumsum(size)[:-1]
    u = rng.uniform(-0.5, 0.5, size=int(size.sum()))
    dist = np.linalg.norm(pos[bj[ks]] + br[ks] @ cell - pos[bi[ks]], axis=1)
    fac = np.exp(-dist / decay)
    onsite = (bi[ks] == bj[ks]) & ~np.any(br[ks] != 0, axis=1)
    for a, b in sorted(set(zip(ni.tolist(), nj.tolist()))):
        sel = np.nonzero((ni == a) & (nj == b))[0]
        blk = u[ustart[sel][:, None] + np.arange(a * b)[None, :]].reshape(-1, a, b) * fac[sel][:, None, None]
        if a == b:
            on = onsite[sel]
            if on.any():
                blk[on] = 0.5 * (blk[on] + np.swapaxes(blk[on], 1, 2)) + np.eye(a)
        k = ks[sel]
        d[off[k][:, None] + np.arange(a * b)[None, :]] = blk.reshape(-1, a * b)
        kt = tr[k]
        d[off[kt][:, None] + np.arange(a * b)[None, :]] = np.swapaxes(blk, 1, 2).reshape(-1, a * b)
    return d


def frac_grid(grid) -> np.ndarray:
    n1, n2, n3 = (int(x) for x in grid)
    s = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3,
                             indexing="ij"), -1)
    return s.reshape(-1, 3)


def plane_wave_potential(grid, millers: np.ndarray, amps: np.ndarray, phases: np.ndarray) -> np.ndarray:
    """V(s_g) = sum_k amp_k cos(2 pi m_k . s_g + phase_k) on the fractional
    grid s_g = n/N, evaluated as the real part of one inverse FFT of the
    sparse coefficient array (the Miller indices must be distinct)."""
    n = tuple(int(x) for x in grid)
    coef = np.zeros(n, dtype=np.complex128)
    for m, a, p in zip(millers, amps, phases):
        idx = tuple(int(m[k]) % n[k] for k in range(3))
        coef[idx] += a * np.exp(1j * p)
    v = np.fft.ifftn(coef).real * float(np.prod(n))
    return np.ascontiguousarray(v.ravel())


def random_millers_box(rng, n_waves: int, mmax: int) -> np.ndarray:
    allm = np.stack(np.meshgrid(*[np.arange(-mmax, mmax + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    allm = allm[np.any(allm != 0, axis=1)]
    sel = rng.choice(allm.shape[0], size=n_waves, replace=False)
    return allm[sel]


def random_millers_gmax(rng, cell, n_waves: int, gmax: float) -> np.ndarray:
    recip = 2.0 * np.pi * np.linalg.inv(cell).T
    nr = np.ceil(gmax / np.linalg.norm(recip, axis=1) * 1.0).astype(int) + 1
    allm = np.stack(np.meshgrid(*[np.arange(-n, n + 1) for n in nr], indexing="ij"), -1).reshape(-1, 3)
    g = np.linalg.norm(allm @ recip, axis=1)
    allm = allm[(g <= gmax) & np.any(allm != 0, axis=1)]
    sel = rng.choice(allm.shape[0], size=min(n_waves, allm.shape[0]), replace=False)
    return allm[sel]


def assemble(cell, pos, species, species_list, grid, v, rng, skin=0.5, name="") -> System:
    species = np.asarray(species, dtype=np.int32)
    norb = np.array([species_list[s].norb for s in species], dtype=np.int64)
    rc = np.array([species_list[s].rcut for s in species], dtype=np.float64)
    bi, bj, br = build_pattern(cell, pos, rc, skin=skin)
    off = block_offsets(bi, bj, norb)
    d = random_density_matrix(cell, pos, bi, bj, br, off, norb, rng)
    nnz = int(d.shape[0])
    return System(cell=np.ascontiguousarray(cell, dtype=np.float64),
                  pos=np.ascontiguousarray(pos, dtype=np.float64), species=species,
                  species_list=list(species_list), grid=np.asarray(grid, dtype=np.int32),
                  blk_i=bi, blk_j=bj, blk_r=np.ascontiguousarray(br), blk_off=off, nnz=nnz,
                  v=np.ascontiguousarray(v), d=d, name=name)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def diamond8(seed: int = 0, grid=(32, 32, 32), rcut: float = 6.0, dr: float = 0.01) -> System:
    """Jittered 8-atom diamond cell, a = 6.74 Bohr, 13 orbitals per C
    (2s2p1d), rcut 6 Bohr, dr 0.01 Bohr, V = 20 plane waves of 0.5 Ha."""
    rng = np.random.default_rng(seed)
    cell, pos = diamond_cell(6.74, 0.05, rng)
    sp = make_species("C", "2s2p1d", rcut, dr, rng)
    millers = random_millers_box(rng, 20, 4)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=20)
    v = plane_wave_potential(grid, millers, np.full(20, 0.5), phases)
    return assemble(cell, pos, np.zeros(8, np.int32), [sp], grid, v, rng, name=f"diamond8_seed{seed}")


def tbg_system(i: int = 8, seed: int = 0, h: float = 0.22, rcut: float = 8.0,
               dr: float = 0.01, a_ang: float = 2.46, vacuum: float = 20.0,
               n_waves: int = 64, gmax: float = 1.5, amp: float = 0.1,
               grid=None) -> System:
    """Twisted bilayer graphene of index i (4(3i^2+3i+1) C atoms), 13
    orbitals per atom, rcut 8 Bohr, grid spacing ~h, V a sum of n_waves
    random plane waves with |G| <= gmax of amplitude amp."""
    rng = np.random.default_rng(seed)
    cell, pos, _ = tbg(i, a_ang=a_ang, vacuum=vacuum)
    sp = make_species("C", "2s2p1d", rcut, dr, rng)
    if grid is None:
        grid = grid_for_spacing(cell, h)
    millers = random_millers_gmax(rng, cell, n_waves, gmax)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=millers.shape[0])
    v = plane_wave_potential(grid, millers, np.full(millers.shape[0], amp), phases)
    return assemble(cell, pos, np.zeros(pos.shape[0], np.int32), [sp], grid, v, rng,
                    name=f"tbg{i}_seed{seed}")


def random_molecular_crystal(seed: int, natom: Optional[int] = None, nmin: int = 40,
                             nmax: int = 600, dr: float = 0.01, min_sep: float = 1.8,
                             vol_per_atom: float = 50.0, h_target: float = 0.32) -> System:
    """Cubic periodic cell of random C/H/O atoms (fractions 0.4/0.4/0.2) with
    a minimum separation; rcut H/C/O = 6/7/8 Bohr; grid clamp(8*round(L/2.56), 32, 96)^3."""
    rng = np.random.default_rng(seed)
    if natom is None:
        natom = int(rng.integers(nmin, nmax + 1))
    L = (vol_per_atom * natom) ** (1.0 / 3.0)
    cell = np.eye(3) * L
    placed = np.zeros((natom, 3))
    n = 0
    tries = 0
    while n < natom:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place atoms")
        p = rng.uniform(0, L, size=3)
        dvec = p[None, :] - placed[:n]
        dvec -= L * np.round(dvec / L)
        if n == 0 or np.min(np.einsum("ij,ij->i", dvec, dvec)) >= min_sep * min_sep:
            placed[n] = p
            n += 1
    pos = placed
    kinds = rng.choice(3, size=natom, p=[0.4, 0.4, 0.2])   # 0=C, 1=H, 2=O
    species_list = [make_species("C", "2s2p1d", 7.0, dr, rng),
                    make_species("H", "2s1p", 6.0, dr, rng),
                    make_species("O", "2s2p1d", 8.0, dr, rng)]
    n = int(min(96, max(32, 8 * round(L / (8 * h_target)))))
    grid = (n, n, n)
    millers = random_millers_box(rng, 20, 3)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=20)
    v = plane_wave_potential(grid, millers, np.full(20, 0.2), phases)
    return assemble(cell, pos, kinds.astype(np.int32), species_list, grid, v, rng,
                    name=f"molcrystal{natom}_seed{seed}")


def molecular_batch(n: int = 64, seed: int = 0, nmin: int = 40, nmax: int = 600) -> list:
    """n independent random C/H/O crystals with atom counts uniform in
    [nmin, nmax] (one seed stream per structure)."""
    return [random_molecular_crystal(seed * 100003 + 17 * i + 1, nmin=nmin, nmax=nmax) for i in range(n)]


def make_config(k: int, seed: int = 0):
    """Named workloads: 1 = jittered diamond (parity), 2 = TBG i=8 (868
    atoms, 3.89 deg), 3 = batch of 64 random C/H/O crystals of 40-600 atoms
    (a list of systems), 5 = TBG i=29 (10,444 atoms, 1.12 deg)."""
    if k == 1:
        return diamond8(seed)
    if k == 2:
        return tbg_system(8, seed)
    if k == 3:
        return molecular_batch(64, seed)
    if k == 5:
        return tbg_system(29, seed)
    raise ValueError(f"unknown config {k}")


def orbital_counts(ls) -> int:
    return int(sum(2 * int(l) + 1 for l in ls))
