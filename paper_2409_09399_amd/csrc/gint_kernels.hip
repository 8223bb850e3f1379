// HIP kernels for grid integration on CDNA4 (gfx950), FP64 path.
//
// Each workgroup (4 waves, 256 threads) takes one work item: a run of
// bigcells (4x4x4 grid points) of one cluster pair (A, B), see
// gint_internal.h.  Per bigcell:
//   phase 1  every thread evaluates orbitals of one A atom and one B atom at
//            one point into LDS tiles phi[point][atom slot][16 orbitals]
//            (cubic Hermite radial table x real solid harmonic, l <= 2), and
//            marks which atoms reach which points;
//   phase 2  MFMA v_mfma_f64_16x16x4f64 contractions on the tiles;
//   phase 3  (rho, force) per-point reductions of the MFMA output.
// Vlocal keeps the 16 (a_i, b_j) output tiles of the pair in registers for
// the whole item (wave i owns row atom a_i) and writes them once at the end.
#include <hip/hip_runtime.h>

#include <mutex>
#include <utility>
#include <vector>

#include "gint_device.h"

typedef double d4 __attribute__((ext_vector_type(4)));

#define PSTR 65     // LDS doubles per point row: 4 slots x 16 orbitals + 1 (bank spread)

namespace {

constexpr double kC0 = 0.28209479177387814;    // 1/(2 sqrt(pi))
constexpr double kC1 = 0.48860251190291992;    // sqrt(3/(4 pi))
constexpr double kC2a = 1.0925484305920792;    // sqrt(15/pi)/2
constexpr double kC2b = 0.31539156525252005;   // sqrt(5/pi)/4
constexpr double kC2c = 0.54627421529603959;   // sqrt(15/pi)/4


__device__ inline int wrap(int n, int N) {
    int m = n % N;
    return m < 0 ? m + N : m;
}

struct Pt {
    double x, y, z;
    long long g;
};

// Point pt (0..63, i-major: i = pt>>4, j = (pt>>2)&3, k = pt&3) of the
// bigcell with origin o.
__device__ inline Pt bigcell_point(const GDev &P, const GBig &o, int pt) {
    const int n0 = o.x + (pt >> 4), n1 = o.y + ((pt >> 2) & 3), n2 = o.z + (pt & 3);
    Pt r;
    r.x = n0 * P.e[0][0] + n1 * P.e[1][0] + n2 * P.e[2][0];
    r.y = n0 * P.e[0][1] + n1 * P.e[1][1] + n2 * P.e[2][1];
    r.z = n0 * P.e[0][2] + n1 * P.e[1][2] + n2 * P.e[2][2];
    if (o.w >= 0)   // the bigcell does not wrap: w is the flat index of its origin
        r.g = o.w + (((pt >> 4) * P.N[1] + ((pt >> 2) & 3)) * P.N[2] + (pt & 3));
    else
        r.g = ((long long)wrap(n0, P.N[0]) * P.N[1] + wrap(n1, P.N[1])) * P.N[2] + wrap(n2, P.N[2]);
    return r;
}

// Hermite basis on [r_k, r_k+1] of the species table; returns the knot row.
struct Herm {
    const double *row0, *row1;
    double h00, h10, h01, h11;     // value weights (h10, h11 include dr)
    double d00, d10, d01, d11;     // derivative weights (per unit r)
};

template <int SHAPE>
__device__ __attribute__((always_inline)) inline Herm hermite(CSpecies &sp, const double *tab, double r) {
    const int nchan = ChanShape<SHAPE>::nchan(sp);
    double t = r * sp.inv_dr;
    int k = (int)t;
    if (k > sp.nknots - 2) k = sp.nknots - 2;
    t -= (double)k;
    const double t2 = t * t, t3 = t2 * t;
    Herm h;
    h.row0 = tab + sp.tab_off + (size_t)k * nchan * 2;
    h.row1 = h.row0 + nchan * 2;
    h.h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
    h.h10 = (t3 - 2.0 * t2 + t) * sp.dr;
    h.h01 = 3.0 * t2 - 2.0 * t3;
    h.h11 = (t3 - t2) * sp.dr;
    h.d00 = (6.0 * t2 - 6.0 * t) * sp.inv_dr;
    h.d10 = 3.0 * t2 - 4.0 * t + 1.0;
    h.d01 = -h.d00;
    h.d11 = 3.0 * t2 - 2.0 * t;
    return h;
}

// The cutoff and table constants of one species, read once per work item
// (a loop over bigcells then issues no species descriptor loads).
struct SpK {
    double rcut2, rcut, inv_dr, dr;
    int kmax;              // last knot interval
    const double *tab0;    // the species' table records
};

// hermite<SHAPE> with the constants of k (the same arithmetic).
__device__ __attribute__((always_inline)) inline Herm hermite_k(const SpK &k, int nchan, double r) {
    double t = r * k.inv_dr;
    int kn = (int)t;
    if (kn > k.kmax) kn = k.kmax;
    t -= (double)kn;
    const double t2 = t * t, t3 = t2 * t;
    Herm h;
    h.row0 = k.tab0 + (size_t)kn * nchan * 2;
    h.row1 = h.row0 + nchan * 2;
    h.h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
    h.h10 = (t3 - 2.0 * t2 + t) * k.dr;
    h.h01 = 3.0 * t2 - 2.0 * t3;
    h.h11 = (t3 - t2) * k.dr;
    h.d00 = (6.0 * t2 - 6.0 * t) * k.inv_dr;
    h.d10 = 3.0 * t2 - 4.0 * t + 1.0;
    h.d01 = -h.d00;
    h.d11 = 3.0 * t2 - 2.0 * t;
    return h;
}

__device__ inline void solid9(double x, double y, double z, double S[9]) {
    S[0] = kC0;
    S[1] = kC1 * y;
    S[2] = kC1 * z;
    S[3] = kC1 * x;
    S[4] = kC2a * x * y;
    S[5] = kC2a * y * z;
    S[6] = kC2b * (2.0 * z * z - x * x - y * y);
    S[7] = kC2a * x * z;
    S[8] = kC2c * (x * x - y * y);
}

// Table values (f, f') of up to RCH channels at knots k and k + 1, all
// loads issued before any is used: a channel loop that loads as it goes
// waits one memory round trip per channel.
constexpr int RCH = 5;
typedef double dbl2 __attribute__((ext_vector_type(2)));

struct Rows {
    dbl2 a[RCH], b[RCH];    // (f_k, f'_k) and (f_k+1, f'_k+1) of channel c0 + q
};

__device__ __attribute__((always_inline)) inline void load_rows(const Herm &h, int nchan, int c0, Rows &R) {
#pragma unroll
    for (int q = 0; q < RCH; ++q)
        if (c0 + q < nchan) {
            R.a[q] = *(const dbl2 *)(h.row0 + 2 * (c0 + q));
            R.b[q] = *(const dbl2 *)(h.row1 + 2 * (c0 + q));
        }
}

// phi_mu(x) * scale for the 16 orbital slots of one atom, written to dst
// (LDS); slots past the atom's orbitals are zero.
template <int SHAPE, bool PAD = true>
__device__ __attribute__((always_inline)) inline void eval_phi_h(CSpecies &sp, const Herm &h, double x, double y,
                                                                 double z, double scale, double *dst) {
    double S[9];
    solid9(x, y, z, S);
    const int nchan = ChanShape<SHAPE>::nchan(sp);
    int slot = 0;
    for (int c0 = 0; c0 < nchan; c0 += RCH) {
        Rows R;
        load_rows(h, nchan, c0, R);
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            if (c0 + q >= nchan) break;
            const double p = (h.h00 * R.a[q].x + h.h10 * R.a[q].y + h.h01 * R.b[q].x + h.h11 * R.b[q].y) * scale;
            const int l = ChanShape<SHAPE>::l(sp, c0 + q);
            if (l == 0) {
                dst[slot] = p * S[0];
                slot += 1;
            } else if (l == 1) {
                dst[slot] = p * S[1];
                dst[slot + 1] = p * S[2];
                dst[slot + 2] = p * S[3];
                slot += 3;
            } else {
                dst[slot] = p * S[4];
                dst[slot + 1] = p * S[5];
                dst[slot + 2] = p * S[6];
                dst[slot + 3] = p * S[7];
                dst[slot + 4] = p * S[8];
                slot += 5;
            }
        }
    }
    // PAD = false leaves the padding slots as they are (where they reach only
    // outputs beyond the orbital count)
    if constexpr (PAD)
        for (; slot < GINT_ORB; ++slot) dst[slot] = 0.0;
}

template <int SHAPE, bool PAD = true>
__device__ __attribute__((always_inline)) inline void eval_phi(CSpecies &sp, const double *tab, double x, double y,
                                                               double z, double r2, double scale, double *dst) {
    eval_phi_h<SHAPE, PAD>(sp, hermite<SHAPE>(sp, tab, sqrt(r2)), x, y, z, scale, dst);
}

__device__ inline void zero16(double *dst) {
#pragma unroll
    for (int k = 0; k < GINT_ORB; ++k) dst[k] = 0.0;
}

// sum_mu psi_mu phi_mu and (GRAD) sum_mu psi_mu grad phi_mu for one atom at
// x (grad phi = (p'/r) x S + p grad S; the first term is 0 at r = 0).
template <bool GRAD, int SHAPE>
__device__ __attribute__((always_inline)) inline void dot_phi(CSpecies &sp, const double *tab, double x, double y,
                                                              double z, double r2, const double *psi, double &e,
                                                              double G[3]) {
    const double r = sqrt(r2);
    const Herm h = hermite<SHAPE>(sp, tab, r);
    const double inv_r = r > 0.0 ? 1.0 / r : 0.0;
    e = 0.0;
    G[0] = G[1] = G[2] = 0.0;
    const int nchan = ChanShape<SHAPE>::nchan(sp);
    int slot = 0;
    for (int c0 = 0; c0 < nchan; c0 += RCH) {
        Rows R;
        load_rows(h, nchan, c0, R);
#pragma unroll
        for (int qq = 0; qq < RCH; ++qq) {
            if (c0 + qq >= nchan) break;
            const double f0 = R.a[qq].x, fp0 = R.a[qq].y, f1 = R.b[qq].x, fp1 = R.b[qq].y;
            const double p = h.h00 * f0 + h.h10 * fp0 + h.h01 * f1 + h.h11 * fp1;
            const double q = GRAD ? (h.d00 * f0 + h.d10 * fp0 + h.d01 * f1 + h.d11 * fp1) * inv_r : 0.0;
            const int l = ChanShape<SHAPE>::l(sp, c0 + qq);
            double A, Bx, By, Bz;   // A = sum_m psi_m S_m, B = sum_m psi_m grad S_m
            if (l == 0) {
                A = psi[slot] * kC0;
                Bx = By = Bz = 0.0;
                slot += 1;
            } else if (l == 1) {
                const double p0 = psi[slot], p1 = psi[slot + 1], p2 = psi[slot + 2];   // (y, z, x)
                A = kC1 * (p0 * y + p1 * z + p2 * x);
                Bx = kC1 * p2;
                By = kC1 * p0;
                Bz = kC1 * p1;
                slot += 3;
            } else {
                const double p0 = psi[slot], p1 = psi[slot + 1], p2 = psi[slot + 2], p3 = psi[slot + 3],
                             p4 = psi[slot + 4];
                A = kC2a * (p0 * x * y + p1 * y * z + p3 * x * z) + kC2b * p2 * (2.0 * z * z - x * x - y * y) +
                    kC2c * p4 * (x * x - y * y);
                Bx = kC2a * (p0 * y + p3 * z) - 2.0 * kC2b * p2 * x + 2.0 * kC2c * p4 * x;
                By = kC2a * (p0 * x + p1 * z) - 2.0 * kC2b * p2 * y - 2.0 * kC2c * p4 * y;
                Bz = kC2a * (p1 * y + p3 * x) + 4.0 * kC2b * p2 * z;
                slot += 5;
            }
            e += p * A;
            if (GRAD) {
                G[0] += q * A * x + p * Bx;
                G[1] += q * A * y + p * By;
                G[2] += q * A * z + p * Bz;
            }
        }
    }
}

__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline unsigned or16(unsigned m) {
    m |= __shfl_xor(m, 1);
    m |= __shfl_xor(m, 2);
    m |= __shfl_xor(m, 4);
    m |= __shfl_xor(m, 8);
    return m;
}

// Phase 1 of rho/force: orbitals of the B atom of slot w at point lane into
// phiB; the A atom of slot w only marks where it is active (the per-point
// phase evaluates it).
template <int KS>
__device__ inline void stage_b(const GDev &P, CPair &pr, const GBig &o, double *phiB, unsigned *maskpt,
                               unsigned *maskt) {
    const int t = threadIdx.x;
    const int pt = t & 63, slot = wave_id();
    const Pt r = bigcell_point(P, o, pt);
    unsigned bits = 0;
    {
        const int a = pr.a[slot];
        bool in = false;
        if (a >= 0) {
            const GAtom at = ldc(P.atoms + (a));
            const double x = r.x - at.x - pr.shiftA[0];
            const double y = r.y - at.y - pr.shiftA[1];
            const double z = r.z - at.z - pr.shiftA[2];
            const double r2 = x * x + y * y + z * z;
            CSpecies &sp = cst(P.species)[at.species];
            in = r2 < sp.rcut2 && sqrt(r2) < sp.rcut;
        }
        if (in) bits |= 1u << slot;
    }
    {
        const int b = pr.b[slot];
        double *dst = phiB + pt * PSTR + slot * GINT_ORB;
        bool in = false;
        double x = 0.0, y = 0.0, z = 0.0, r2 = 0.0;
        int species = 0;
        if (b >= 0) {
            const GAtom at = ldc(P.atoms + (b));
            x = r.x - at.x - pr.shiftB[0];
            y = r.y - at.y - pr.shiftB[1];
            z = r.z - at.z - pr.shiftB[2];
            r2 = x * x + y * y + z * z;
            species = at.species;
            CSpecies &sp = cst(P.species)[species];
            in = r2 < sp.rcut2 && sqrt(r2) < sp.rcut;
        }
        // with the per-tile masks the psi products skip a B atom on 16-point
        // tiles where it is inactive, so zeros go only into tiles where it is
        // active somewhere (ballot taken by the whole wave)
        const unsigned long long act = __ballot(in);
        if (in) {
            CSpecies &sp = cst(P.species)[species];
            with_shape<KS>(sp, [&](auto shp) {
                eval_phi<decltype(shp)::value>(sp, P.tab, x, y, z, r2, 1.0, dst);
            });
            bits |= 1u << (4 + slot);
        } else if ((act >> (pt & ~15)) & 0xFFFFull) {
            zero16(dst);
        }
    }
    if (bits) atomicOr(&maskpt[pt], bits);
    // activity per 16-point tile, packed in one word (tile t: bit 8t + slot
    // for A, 8t + 4 + slot for B) from the wave's ballots: one atomic per wave
    const unsigned long long ba = __ballot((bits >> slot) & 1u), bb = __ballot(bits >> 4);
    unsigned tw = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if ((ba >> (16 * q)) & 0xFFFFull) tw |= 1u << (8 * q + slot);
        if ((bb >> (16 * q)) & 0xFFFFull) tw |= 1u << (8 * q + 4 + slot);
    }
    if (pt == 0 && tw) atomicOr(maskt, tw);
}

// Row atom i of D_sym as MFMA B operands: dw[j][s] holds
// D_sym[a_i mu][b_j nu] with mu = lane & 15, nu = 4 s + (lane >> 4).
__device__ inline void load_dsym_row(const GDev &P, CPair &pr, const double *__restrict__ D, int i,
                                     double dw[4][4]) {
    const int lane = threadIdx.x & 63;
    const int mu = lane & 15;
    const int na = pr.a[i] >= 0 ? cst(P.atoms)[pr.a[i]].norb : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const long long o = pr.hoff[i * 4 + j], ot = pr.hoff_t[i * 4 + j];
        const int nb = pr.b[j] >= 0 ? cst(P.atoms)[pr.b[j]].norb : 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int nu = 4 * s + (lane >> 4);
            double v = 0.0;
            if (o >= 0 && ot >= 0 && mu < na && nu < nb)
                v = 0.5 * (D[o + (long long)mu * nb + nu] + D[ot + (long long)nu * na + mu]);
            dw[j][s] = v;
        }
    }
}

// Phase 2 of rho/force: wave w computes psi[pt][mu] = sum_{b_j, nu}
// phi_B[pt][b_j][nu] D_sym[a_w mu][b_j nu] for all 64 points (four 16-point
// tiles; tiles where a_w is inactive are skipped, and B atoms inactive on a
// tile are skipped).  Result in registers, MFMA layout: c[t] lane l register
// q holds point 16 t + 4 q + (l >> 4), orbital l & 15.
__device__ inline void psi_row(const double dw[4][4], const double *phiB, const unsigned *maskt, d4 c[4]) {
    const int lane = threadIdx.x & 63, w = wave_id();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        c[t] = (d4){0.0, 0.0, 0.0, 0.0};
        const unsigned gm = (__builtin_amdgcn_readfirstlane(*maskt) >> (8 * t)) & 0xFFu;
        if (!(gm & (1u << w))) continue;
        const double *base = phiB + (16 * t + (lane & 15)) * PSTR + (lane >> 4);
        // operands only of B atoms active on the tile (their zeros are written
        // only there)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!(gm & (1u << (4 + j)))) continue;
            double src[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) src[s] = base[j * GINT_ORB + 4 * s];
#pragma unroll
            for (int s = 0; s < 4; ++s) c[t] = mfma64(src[s], dw[j][s], c[t]);
        }
    }
}

// Store psi of atom slot w over that slot's columns of phiB (after every
// wave has finished reading phiB); only rows of tiles where a_w is active.
__device__ inline void store_psi(const d4 c[4], double *phiB, const unsigned *maskt) {
    const int lane = threadIdx.x & 63, w = wave_id();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const unsigned gm = (__builtin_amdgcn_readfirstlane(*maskt) >> (8 * t)) & 0xFFu;
        if (!(gm & (1u << w))) continue;
        double *dst = phiB + (16 * t + (lane >> 4)) * PSTR + w * GINT_ORB + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[4 * q * PSTR] = c[t][q];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// H_IJR (Eq. 2), FP64.  Eight waves share the two 64-point tiles: wave w
// evaluates one orbital set (A for w < 4, B scaled by w V_g for w >= 4, slot
// w & 3) and, in the contraction, owns row atom a_i (i = w & 3) over the 32
// points of half h = w >> 2, accumulating the four (a_i, b_j) tiles of those
// points.  The two halves are added through LDS when the item ends and each
// block is written once (plain stores when the item covers the whole pair,
// atomics otherwise), with its transpose (b_j, a_i, -R).  With the LDS of the
// tiles the limit, eight waves per workgroup double the waves per CU of a
// four-wave layout.
// ---------------------------------------------------------------------------
constexpr int kVlocalThreads = 512;

// The atom image of one slot of a work item and its species' constants,
// read once per item.  species < 0: empty slot.
struct SlotK {
    double ax, ay, az, sx, sy, sz;    // atom position and lattice shift of the image
    int species;
    SpK k;
};

__device__ inline SlotK slot_k(const GDev &P, int a, cdouble *sh) {
    SlotK s{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1, SpK{0.0, 0.0, 0.0, 0.0, 0, P.tab}};
    if (a >= 0) {
        const GAtom at = ldc(P.atoms + a);
        CSpecies &sp = cst(P.species)[at.species];
        s = SlotK{at.x, at.y, at.z, sh[0], sh[1], sh[2], at.species,
                  SpK{sp.rcut2, sp.rcut, sp.inv_dr, sp.dr, sp.nknots - 2, P.tab + sp.tab_off}};
    }
    return s;
}

template <int KS>
__device__ inline void stage_vlocal(const GDev &P, const SlotK &sk, const GBig &o, const double *__restrict__ V,
                                    double *phiA, double *phiB, unsigned *maskpt) {
    const int pt = threadIdx.x & 63, w = wave_id();
    const int slot = w & 3;
    const bool sideB = w >= 4;
    const Pt r = bigcell_point(P, o, pt);
    // B waves request V first, so its latency overlaps the displacement work
    const double vpt = sideB ? V[r.g] : 0.0;
    double *dst = (sideB ? phiB : phiA) + pt * PSTR + slot * GINT_ORB;
    bool in = false;
    double x = 0.0, y = 0.0, z = 0.0, r2 = 0.0;
    if (sk.species >= 0) {
        x = r.x - sk.ax - sk.sx;
        y = r.y - sk.ay - sk.sy;
        z = r.z - sk.az - sk.sz;
        r2 = x * x + y * y + z * z;
        in = r2 < sk.k.rcut2 && sqrt(r2) < sk.k.rcut;
    }
    // zeros only where they are read: a 4-point k-step of this slot enters
    // the products only if the slot is active at one of its points (ballot
    // taken by the whole wave)
    const unsigned long long act = __ballot(in);
    if (in) {
        CSpecies &sp = cst(P.species)[sk.species];
        // with a fixed layout the padding rows are not stored: they reach only
        // output rows or columns beyond the orbital count, which are never written
        with_shape<KS>(sp, [&](auto shp) {
            constexpr int SH = decltype(shp)::value;
            eval_phi_h<SH, KS == GINT_SHAPE_ANY>(sp, hermite_k(sk.k, ChanShape<SH>::nchan(sp), sqrt(r2)), x, y, z,
                                                 sideB ? P.w * vpt : 1.0, dst);
        });
        atomicOr(&maskpt[pt], 1u << (sideB ? 4 + slot : slot));
    } else if ((act >> (pt & ~3)) & 0xFull) {
        if constexpr (KS == GINT_SHAPE_ANY) {
            zero16(dst);
        } else {
#pragma unroll
            for (int k = 0; k < ChanShape<KS>::norb; ++k) dst[k] = 0.0;
        }
    }
}

template <int KS>
__global__ __launch_bounds__(kVlocalThreads, 4) void k_vlocal(GDev P0, const double *__restrict__ V0,
                                                              double *__restrict__ H) {
    __shared__ double phiA[GINT_BCPTS * PSTR];
    __shared__ double phiB[GINT_BCPTS * PSTR];
    __shared__ unsigned maskpt[GINT_BCPTS];
    __shared__ int s_item;
    for (;;) {
    const int item_ = claim_item(P0.counter, &s_item);
    if (item_ >= P0.nitems) break;
    const GItem it = ldc(P0.items + item_);
    CPair &pr = cst(P0.pairs)[it.pair];
    GDev P = P0;
    bind_system(P, pr.sys);
    CSys &SY = cst(P0.sys)[pr.sys];
    const double *V = V0 + SY.g_off;
    const int lane = threadIdx.x & 63, w = wave_id();
    const int i = w & 3, half = w >> 2;
    const SlotK sk = slot_k(P, half ? pr.b[i] : pr.a[i], half ? pr.shiftB : pr.shiftA);
    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};

    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        if (threadIdx.x < GINT_BCPTS) maskpt[threadIdx.x] = 0u;
        __syncthreads();
        stage_vlocal<KS>(P, sk, o, V, phiA, phiB, maskpt);
        __syncthreads();
        // k-step t of this wave = points 32 half + 4t .. +3; its activity mask is
        // the OR over those 4 points, read into scalar registers once
        const unsigned mp = maskpt[32 * half + (lane & 31)];
        unsigned mk = mp | __shfl_xor(mp, 1);
        mk |= __shfl_xor(mk, 2);
        unsigned km[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) km[t] = __builtin_amdgcn_readlane(mk, 4 * t);
        const int row0 = (32 * half + (lane >> 4)) * PSTR + (lane & 15);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (!(km[t] & (1u << i))) continue;
            const double a = phiA[row0 + 4 * t * PSTR + i * GINT_ORB];
            // B operands only of atoms active in this k-step (their zeros are
            // written only there)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (km[t] & (1u << (4 + j))) acc[j] = mfma64(a, phiB[row0 + 4 * t * PSTR + j * GINT_ORB], acc[j]);
        }
        __syncthreads();
    }
    // the second half's partial tiles go through LDS ([wave][j][q][lane], 4096
    // doubles in phiA); the first half adds them and writes its row's blocks
    double *red = phiA;
    if (half == 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[((i * 4 + j) * 4 + q) * 64 + lane] = acc[j][q];
    }
    __syncthreads();
    const int ai = pr.a[i];
    if (half == 0 && ai >= 0) {
        const bool exclusive = it.pad != 0;
        const int na = cst(P.atoms)[ai].norb;
        const int nu = lane & 15;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int bj = pr.b[j];
            if (bj < 0) continue;
            const int nb = cst(P.atoms)[bj].norb;
            const long long off = pr.hoff[i * 4 + j], offt = pr.hoff_t[i * 4 + j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // 16x16x4 FP64 result layout: lane l, register q holds row 4q + (l >> 4), column l & 15
                const int mu = 4 * q + (lane >> 4);
                if (mu >= na || nu >= nb) continue;
                const double v = acc[j][q] + red[((i * 4 + j) * 4 + q) * 64 + lane];
                if (exclusive) {
                    if (off >= 0) H[off + (long long)mu * nb + nu] = v;
                    if (!pr.self && offt >= 0) H[offt + (long long)nu * na + mu] = v;
                } else {
                    if (off >= 0) atomicAdd(H + off + (long long)mu * nb + nu, v);
                    if (!pr.self && offt >= 0) atomicAdd(H + offt + (long long)nu * na + mu, v);
                }
            }
        }
    }
    }
}

// ---------------------------------------------------------------------------
// rho_g (Eq. 3): canonical pairs, weight 2 off the self pair.  Wave w owns A
// atom slot w: psi of a_w for the 64 points by MFMA, then per point (lane)
// phi_{a_w} . psi evaluated on the fly.
// ---------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(256, 4) void k_rho(GDev P0, const double *__restrict__ D, double *__restrict__ rho0) {
    __shared__ double phiB[GINT_BCPTS * PSTR];
    __shared__ unsigned maskpt[2][GINT_BCPTS];
    __shared__ unsigned maskt[2];
    __shared__ int s_item;
    // masks are double-buffered: each bigcell uses buffer cur, which is clear
    // on entry, and clears the other one for the next bigcell
    if (threadIdx.x < 2 * GINT_BCPTS) maskpt[threadIdx.x >> 6][threadIdx.x & 63] = 0u;
    if (threadIdx.x < 2) maskt[threadIdx.x] = 0u;
    int cur = 0;
    for (;;) {
    const int item_ = claim_item(P0.counter, &s_item);
    if (item_ >= P0.nitems) break;
    const GItem it = ldc(P0.items + item_);
    CPair &pr = cst(P0.pairs)[it.pair];
    GDev P = P0;
    bind_system(P, pr.sys);
    CSys &SY = cst(P0.sys)[pr.sys];
    double *rho = rho0 + SY.g_off;
    const int lane = threadIdx.x & 63, w = wave_id();
    const int aw = pr.a[w];
    double dw[4][4];
    load_dsym_row(P, pr, D, w, dw);
    const double weight = pr.self ? 1.0 : 2.0;

    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        unsigned *mpt = maskpt[cur], *mt = &maskt[cur];
        stage_b<KS>(P, pr, o, phiB, mpt, mt);
        __syncthreads();
        // the other buffer was last read before the previous bigcell's final barrier
        if (threadIdx.x < GINT_BCPTS) maskpt[cur ^ 1][threadIdx.x] = 0u;
        if (threadIdx.x == GINT_BCPTS) maskt[cur ^ 1] = 0u;
        cur ^= 1;
        d4 c[4];
        psi_row(dw, phiB, mt, c);
        __syncthreads();
        store_psi(c, phiB, mt);
        // phase 3: wave w = A slot w, lane = point (reads only its own psi)
        {
            double v = 0.0;
            if (aw >= 0 && (mpt[lane] & (1u << w)) && (mpt[lane] & 0xF0u)) {   // psi is 0 where no B atom reaches
                const Pt r = bigcell_point(P, o, lane);
                const GAtom at = ldc(P.atoms + aw);
                const double x = r.x - at.x - pr.shiftA[0];
                const double y = r.y - at.y - pr.shiftA[1];
                const double z = r.z - at.z - pr.shiftA[2];
                double G[3];
                CSpecies &spa = cst(P.species)[at.species];
                with_shape<KS>(spa, [&](auto shp) {
                    dot_phi<false, decltype(shp)::value>(spa, P.tab, x, y, z, x * x + y * y + z * z,
                                                         phiB + lane * PSTR + w * GINT_ORB, v, G);
                });
                // each wave adds its atom's term: no LDS sum over the waves and
                // no barrier for it, at the price of more atomics
                atomicAdd(rho + r.g, weight * v);
            }
        }
        __syncthreads();
    }
    }
}

// ---------------------------------------------------------------------------
// Pulay force and strain derivative (Eq. 4-5): ordered pairs, A side only.
// Wave w owns A atom slot w (psi by MFMA, then grad phi . psi per point).
// With RHO the per-point values phi_A . psi_A, which the energy needs anyway,
// are also added into rho: over the two orders of a pair they give rho's
// weight 2 off the self pair, so one pass yields rho, F, Z and E.
// ---------------------------------------------------------------------------
template <bool RHO, int KS>
__global__ __launch_bounds__(256, 3) void k_force(GDev P0, const double *__restrict__ V0,
                                                  const double *__restrict__ D, double *__restrict__ F,
                                                  double *__restrict__ ZE0, double *__restrict__ rho0) {
    __shared__ double phiB[GINT_BCPTS * PSTR];
    __shared__ unsigned maskpt[2][GINT_BCPTS];
    __shared__ unsigned maskt[2];
    __shared__ double red[4][10];
    __shared__ int s_item;
    // masks are double-buffered: each bigcell uses buffer cur, which is clear
    // on entry, and clears the other one for the next bigcell
    if (threadIdx.x < 2 * GINT_BCPTS) maskpt[threadIdx.x >> 6][threadIdx.x & 63] = 0u;
    if (threadIdx.x < 2) maskt[threadIdx.x] = 0u;
    int cur = 0;
    for (;;) {
    const int item_ = claim_item(P0.counter, &s_item);
    if (item_ >= P0.nitems) break;
    const GItem it = ldc(P0.items + item_);
    CPair &pr = cst(P0.pairs)[it.pair];
    GDev P = P0;
    bind_system(P, pr.sys);
    CSys &SY = cst(P0.sys)[pr.sys];
    const double *V = V0 + SY.g_off;
    double *ZE = ZE0 + 10 * pr.sys;
    double *rho = RHO ? rho0 + SY.g_off : nullptr;
    const int lane = threadIdx.x & 63, w = wave_id();
    const int aw = pr.a[w];
    double dw[4][4];
    load_dsym_row(P, pr, D, w, dw);
    double f[3] = {0, 0, 0}, z[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, en = 0.0;

    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        unsigned *mpt = maskpt[cur], *mt = &maskt[cur];
        const long long gl = bigcell_point(P, o, lane).g;
        const double vpt = V[gl];   // requested early: its latency overlaps the stage
        stage_b<KS>(P, pr, o, phiB, mpt, mt);
        __syncthreads();
        // the other buffer was last read before the previous bigcell's final barrier
        if (threadIdx.x < GINT_BCPTS) maskpt[cur ^ 1][threadIdx.x] = 0u;
        if (threadIdx.x == GINT_BCPTS) maskt[cur ^ 1] = 0u;
        cur ^= 1;
        d4 c[4];
        psi_row(dw, phiB, mt, c);
        __syncthreads();
        store_psi(c, phiB, mt);
        double e = 0.0;
        if (aw >= 0 && (mpt[lane] & (1u << w)) && (mpt[lane] & 0xF0u)) {   // psi is 0 where no B atom reaches
            const Pt r = bigcell_point(P, o, lane);
            const GAtom at = ldc(P.atoms + aw);
            const double x = r.x - at.x - pr.shiftA[0];
            const double y = r.y - at.y - pr.shiftA[1];
            const double zz = r.z - at.z - pr.shiftA[2];
            const double r2 = x * x + y * y + zz * zz;
            double G[3];
            CSpecies &spa = cst(P.species)[at.species];
            with_shape<KS>(spa, [&](auto shp) {
                dot_phi<true, decltype(shp)::value>(spa, P.tab, x, y, zz, r2, phiB + lane * PSTR + w * GINT_ORB, e, G);
            });
            const double wv = P.w * vpt;
            const double c2 = 2.0 * wv;
            f[0] += c2 * G[0];
            f[1] += c2 * G[1];
            f[2] += c2 * G[2];
            const double xs[3] = {x, y, zz};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) z[3 * a + b] += c2 * G[a] * xs[b];
            en += wv * e;
        }
        // each wave adds its atom's rho term (over the two orders of a pair this
        // gives rho's weight 2 off the self pair)
        if (RHO && e != 0.0) atomicAdd(rho + gl, e);
        __syncthreads();
    }
    // reduce over the wave
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] += __shfl_xor(f[a], off);
#pragma unroll
        for (int a = 0; a < 9; ++a) z[a] += __shfl_xor(z[a], off);
        en += __shfl_xor(en, off);
    }
    if (lane == 0) {
        if (aw >= 0) {
            atomicAdd(F + 3 * aw + 0, f[0]);
            atomicAdd(F + 3 * aw + 1, f[1]);
            atomicAdd(F + 3 * aw + 2, f[2]);
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) red[w][a] = z[a];
        red[w][9] = en;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        const int k = threadIdx.x;
        atomicAdd(ZE + k, red[0][k] + red[1][k] + red[2][k] + red[3][k]);
    }
    }
}

// ---------------------------------------------------------------------------
// W = sum_g n_orb(g)^2 from the canonical pairs (exact in FP64: integers)
// ---------------------------------------------------------------------------
template <int CL>
__global__ __launch_bounds__(256) void k_work(GDev P0, double *__restrict__ W0) {
    __shared__ double red[256];
    __shared__ int s_item;
    const GPairT<CL> *pairs;
    if constexpr (CL == GINT_CL8)
        pairs = P0.pairs8;
    else
        pairs = P0.pairs;
    for (;;) {
    const int item_ = claim_item(P0.counter, &s_item);
    if (item_ >= P0.nitems) break;
    const GItem it = ldc(P0.items + item_);
    const __attribute__((address_space(4))) GPairT<CL> &pr = cst(pairs)[it.pair];
    GDev P = P0;
    bind_system(P, pr.sys);
    CSys &SY = cst(P0.sys)[pr.sys];
    double *W = W0 + pr.sys;
    const double weight = pr.self ? 1.0 : 2.0;
    double acc = 0.0;
    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        if (threadIdx.x < GINT_BCPTS) {
            const Pt r = bigcell_point(P, o, threadIdx.x);
            double na = 0, nb = 0;
            for (int k = 0; k < CL; ++k) {
                if (pr.a[k] >= 0) {
                    const GAtom at = ldc(P.atoms + pr.a[k]);
                    const double x = r.x - at.x - pr.shiftA[0], y = r.y - at.y - pr.shiftA[1],
                                 z = r.z - at.z - pr.shiftA[2];
                    const double r2 = x * x + y * y + z * z;
                    CSpecies &sp = cst(P.species)[at.species];
                    if (r2 < sp.rcut2 && sqrt(r2) < sp.rcut) na += at.norb;
                }
                if (pr.b[k] >= 0) {
                    const GAtom at = ldc(P.atoms + pr.b[k]);
                    const double x = r.x - at.x - pr.shiftB[0], y = r.y - at.y - pr.shiftB[1],
                                 z = r.z - at.z - pr.shiftB[2];
                    const double r2 = x * x + y * y + z * z;
                    CSpecies &sp = cst(P.species)[at.species];
                    if (r2 < sp.rcut2 && sqrt(r2) < sp.rcut) nb += at.norb;
                }
            }
            acc += weight * na * nb;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(W, red[0]);
    }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_fill(double *__restrict__ p, long long n, double v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Largest |D_IJR[mu,nu] - D_JI(-R)[nu,mu]| per system: the symmetry the
// kernels assume when they use D_sym (one block per thread; the maximum of
// non-negative doubles is taken on their bit patterns, which order the same
// way; a NaN difference reports as NaN).
__global__ __launch_bounds__(256) void k_dsym_check(const GBlk *__restrict__ blk, long long nblk,
                                                    const double *__restrict__ D,
                                                    unsigned long long *__restrict__ out) {
    for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < nblk;
         b += (long long)gridDim.x * blockDim.x) {
        const GBlk k = blk[b];
        double m = 0.0;
        for (int mu = 0; mu < k.ni; ++mu)
            for (int nu = 0; nu < k.nj; ++nu) {
                const double d = fabs(D[k.off + (long long)mu * k.nj + nu] - D[k.off_t + (long long)nu * k.ni + mu]);
                m = (d > m || d != d) ? d : m;
            }
        if (m != 0.0) atomicMax(out + k.sys, (unsigned long long)__double_as_longlong(m));
    }
}

// Per-system sums of w_s * x (or w_s * x * y when y is given) over each
// system's grid range (two passes, deterministic): part[s * nparts + b] then
// out[s].
__global__ __launch_bounds__(256) void k_seg_sum_partial(GDev P, const double *__restrict__ x,
                                                         const double *__restrict__ y, int nparts,
                                                         double *__restrict__ part) {
    __shared__ double red[256];
    CSys &S = cst(P.sys)[blockIdx.y];
    const long long n = (long long)S.N[0] * S.N[1] * S.N[2];
    const double *xs = x + S.g_off;
    double acc = 0.0;
    if (y) {
        const double *ys = y + S.g_off;
        for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
            acc += xs[i] * ys[i];
    } else {
        for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) acc += xs[i];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)blockIdx.y * nparts + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_seg_sum_final(GDev P, const double *__restrict__ part, int nparts,
                                                       double *__restrict__ out) {
    __shared__ double red[256];
    const int sy = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[(long long)sy * nparts + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[sy] = red[0] * cst(P.sys)[sy].w;
}

// stress_s = -Z_s / Omega_s, energy_s = E_s
__global__ void k_finish_stress(GDev P, const double *__restrict__ ZE, double *__restrict__ stress,
                                double *__restrict__ energy) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int sy = t / 10, k = t % 10;
    if (sy >= P.nsys) return;
    if (k < 9) stress[9 * sy + k] = -ZE[10 * sy + k] / cst(P.sys)[sy].volume;
    else if (energy) energy[sy] = ZE[10 * sy + 9];
}

// ---------------------------------------------------------------------------
// launchers (called from the C ABI layer)
// ---------------------------------------------------------------------------
// Resident workgroups per device for a kernel (CUs x occupancy), cached so
// that launches inside a stream capture make no device queries.
namespace {
struct GridKey {
    const void *kernel;
    int device;
};
std::mutex g_grid_mu;
std::vector<std::pair<GridKey, int>> g_grid_cache;
}  // namespace

int gint_resident_blocks(const void *kernel, int threads) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    {
        std::lock_guard<std::mutex> lk(g_grid_mu);
        for (const auto &e : g_grid_cache)
            if (e.first.kernel == kernel && e.first.device == dev) return e.second;
    }
    int cus = 0, per_cu = 0;
    if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    const int slots = cus * per_cu;
    std::lock_guard<std::mutex> lk(g_grid_mu);
    g_grid_cache.push_back({GridKey{kernel, dev}, slots});
    return slots;
}

int gint_persistent_grid(const void *kernel, int nitems, int threads) {
    const int slots = gint_resident_blocks(kernel, threads);
    return nitems < slots ? nitems : slots;
}

hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Reset the work counter, then one persistent launch over all items.
#define GINT_PERSISTENT_LAUNCH_T(KERNEL, THREADS, P, s, ...)                                         \
    do {                                                                                            \
        if ((P).nitems <= 0) return hipSuccess;                                                     \
        hipError_t e_ = gint_launch_fill((double *)(P).counter, 1, 0.0, s);                         \
        if (e_ != hipSuccess) return e_;                                                            \
        const int grid_ = gint_persistent_grid((const void *)KERNEL, (P).nitems, THREADS);          \
        hipLaunchKernelGGL(KERNEL, dim3(grid_), dim3(THREADS), 0, s, P, __VA_ARGS__);               \
        return hipGetLastError();                                                                   \
    } while (0)
#define GINT_PERSISTENT_LAUNCH(KERNEL, P, s, ...) GINT_PERSISTENT_LAUNCH_T(KERNEL, 256, P, s, __VA_ARGS__)

hipError_t gint_launch_vlocal(const GDev &P, const double *V, double *H, hipStream_t s) {
    if (P.shape_all == GINT_SHAPE_2S2P1D) {
        auto k = k_vlocal<GINT_SHAPE_2S2P1D>;
        GINT_PERSISTENT_LAUNCH_T(k, kVlocalThreads, P, s, V, H);
    }
    auto k = k_vlocal<GINT_SHAPE_ANY>;
    GINT_PERSISTENT_LAUNCH_T(k, kVlocalThreads, P, s, V, H);
}

hipError_t gint_launch_rho(const GDev &P, const double *D, double *rho, hipStream_t s) {
    if (P.shape_all == GINT_SHAPE_2S2P1D) {
        auto k = k_rho<GINT_SHAPE_2S2P1D>;
        GINT_PERSISTENT_LAUNCH(k, P, s, D, rho);
    }
    auto k = k_rho<GINT_SHAPE_ANY>;
    GINT_PERSISTENT_LAUNCH(k, P, s, D, rho);
}

hipError_t gint_launch_force(const GDev &P, const double *V, const double *D, double *F, double *ZE, double *rho,
                             hipStream_t s) {
    const bool fixed = P.shape_all == GINT_SHAPE_2S2P1D;
    if (rho) {
        auto k = fixed ? k_force<true, GINT_SHAPE_2S2P1D> : k_force<true, GINT_SHAPE_ANY>;
        GINT_PERSISTENT_LAUNCH(k, P, s, V, D, F, ZE, rho);
    }
    auto k = fixed ? k_force<false, GINT_SHAPE_2S2P1D> : k_force<false, GINT_SHAPE_ANY>;
    GINT_PERSISTENT_LAUNCH(k, P, s, V, D, F, ZE, (double *)nullptr);
}

hipError_t gint_launch_work(const GDev &P, double *W, hipStream_t s) {
    if (P.pairs8) GINT_PERSISTENT_LAUNCH(k_work<GINT_CL8>, P, s, W);
    GINT_PERSISTENT_LAUNCH(k_work<GINT_CL>, P, s, W);
}

hipError_t gint_launch_dsym_check(const GBlk *blk, long long nblk, const double *D, double *out, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    const long long nb = (nblk + 255) / 256;
    hipLaunchKernelGGL(k_dsym_check, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, s, blk, nblk, D,
                       reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t gint_launch_seg_sum(const GDev &P, const double *x, const double *y, double *part, int nparts,
                               double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_sum_partial, dim3(nparts, P.nsys), dim3(256), 0, s, P, x, y, nparts, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_sum_final, dim3(P.nsys), dim3(256), 0, s, P, part, nparts, out);
    return hipGetLastError();
}

hipError_t gint_launch_finish_stress(const GDev &P, const double *ZE, double *stress, double *energy,
                                     hipStream_t s) {
    const int n = 10 * P.nsys;
    hipLaunchKernelGGL(k_finish_stress, dim3((n + 255) / 256), dim3(256), 0, s, P, ZE, stress, energy);
    return hipGetLastError();
}

// Fill the resident-block cache for every kernel of a precision form.
void gint_prime_grids_fp64() {
    gint_resident_blocks((const void *)k_vlocal<GINT_SHAPE_ANY>, kVlocalThreads);
    gint_resident_blocks((const void *)k_vlocal<GINT_SHAPE_2S2P1D>, kVlocalThreads);
    gint_resident_blocks((const void *)k_rho<GINT_SHAPE_ANY>, 256);
    gint_resident_blocks((const void *)k_rho<GINT_SHAPE_2S2P1D>, 256);
    gint_resident_blocks((const void *)k_force<false, GINT_SHAPE_ANY>, 256);
    gint_resident_blocks((const void *)k_force<false, GINT_SHAPE_2S2P1D>, 256);
    gint_resident_blocks((const void *)k_force<true, GINT_SHAPE_ANY>, 256);
    gint_resident_blocks((const void *)k_force<true, GINT_SHAPE_2S2P1D>, 256);
    gint_resident_blocks((const void *)k_work<GINT_CL>, 256);
    gint_resident_blocks((const void *)k_work<GINT_CL8>, 256);
}
