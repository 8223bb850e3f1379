// Device helpers of the mixed-precision kernels (FP32 orbitals from FP32
// cubic radial tables, 16-bit hi/lo operand splits, FP16/BF16 MFMA), shared
// by the cluster-pair kernels (gint_kernels_mixed.hip) and the
// bigcell-stationary ones (gint_kernels_bc.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "gint_device.h"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef float flt4_t __attribute__((ext_vector_type(4)));

namespace {

// The FP32 radial tables carry each channel's solid-harmonic normalisation
// K_l (see the plan builder), so the angular factors here are the plain
// polynomials y, z, x (l = 1) and xy, yz, Q (2z^2 - x^2 - y^2), xz,
// (x^2 - y^2)/2 (l = 2).  Q = 1/(2 sqrt 3) is the ratio of the m = 0
// constant to K_2; it enters as an unevaluated FP32 pair (Q = kQh + kQl to
// ~2^-48), so that its own rounding adds no bias.
constexpr float kQh = 0.28867513459481287f;
constexpr float kQl = (float)(0.28867513459481287 - (double)0.28867513459481287f);

__device__ inline float mulQ(float u) { return fmaf(u, kQh, u * kQl); }

// Pins v to its FP32 value in a register.  The hi/lo split needs hi + lo to
// reproduce that value; without the pin the compiler may fuse the product
// that produced v into the two conversions differently (hi from the product
// rounded to FP32, lo from the exact product, each rounded once to 16 bits),
// and where those roundings differ hi + lo misses v by a 16-bit ulp.
__device__ inline void fp32_value(float &v) { asm("" : "+v"(v)); }

template <class T>
struct Split16;

// FP16: lo comes from one mixed-precision FMA, -hi * 1 + v with hi read as
// FP16, rounded once to FP16.  v - hi is exact in FP32 (hi is v rounded to
// 11 bits, so the difference needs at most 12), hence this gives the same
// bits as converting hi back, subtracting and rounding, in one instruction
// instead of three.
template <>
struct Split16<_Float16> {
    typedef h8v vec;
    static constexpr bool pairs = true;
    __device__ static inline void split(float v, _Float16 &hi, _Float16 &lo) {
        fp32_value(v);
        hi = (_Float16)v;
        lo = (_Float16)(v - (float)hi);
    }
    // the same with the one-instruction lo (used where the kernel instance has
    // a fixed channel layout; in the per-species instances the inline asm
    // costs register spills)
    __device__ static inline void split_mix(float v, _Float16 &hi, _Float16 &lo) {
        fp32_value(v);
        hi = (_Float16)v;
        unsigned l;
        asm("v_fma_mixlo_f16 %0, -%1, %3, %2 op_sel_hi:[1,0,0]" : "=v"(l) : "v"(hi), "v"(v), "s"(1.0f));
        lo = __builtin_bit_cast(_Float16, (unsigned short)l);
    }
    // two values as packed pairs (the first in the low half): one packed
    // conversion for hi and the lo halves written in place
    __device__ static inline void split2(float v0, float v1, unsigned &hi, unsigned &lo) {
        fp32_value(v0);
        fp32_value(v1);
        asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(hi) : "v"(v0), "v"(v1));
        asm("v_fma_mixlo_f16 %0, -%1, %4, %2 op_sel_hi:[1,0,0]\n\t"
            "v_fma_mixhi_f16 %0, -%1, %4, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
            : "=&v"(lo) : "v"(hi), "v"(v0), "v"(v1), "s"(1.0f));
    }
    __device__ static inline f4v mfma(vec a, vec b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Split16<__bf16> {
    typedef b8v vec;
    static constexpr bool pairs = false;
    __device__ static inline void split(float v, __bf16 &hi, __bf16 &lo) {
        fp32_value(v);
        hi = (__bf16)v;
        lo = (__bf16)(v - (float)hi);
    }
    __device__ static inline void split_mix(float v, __bf16 &hi, __bf16 &lo) { split(v, hi, lo); }
    __device__ static inline f4v mfma(vec a, vec b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};


__device__ inline int wrapi(int n, int N) {
    int m = n % N;
    return m < 0 ? m + N : m;
}

struct P3 {
    double x, y, z;
    long long g;
};

__device__ inline P3 point_of(const GDev &P, const GBig &o, int pt) {
    const int n0 = o.x + (pt >> 4), n1 = o.y + ((pt >> 2) & 3), n2 = o.z + (pt & 3);
    P3 r;
    r.x = n0 * P.e[0][0] + n1 * P.e[1][0] + n2 * P.e[2][0];
    r.y = n0 * P.e[0][1] + n1 * P.e[1][1] + n2 * P.e[2][1];
    r.z = n0 * P.e[0][2] + n1 * P.e[1][2] + n2 * P.e[2][2];
    if (o.w >= 0)   // the bigcell does not wrap: w is the flat index of its origin
        r.g = o.w + (((pt >> 4) * P.N[1] + ((pt >> 2) & 3)) * P.N[2] + (pt & 3));
    else
        r.g = ((long long)wrapi(n0, P.N[0]) * P.N[1] + wrapi(n1, P.N[1])) * P.N[2] + wrapi(n2, P.N[2]);
    return r;
}

// Workgroup barrier ordering LDS traffic only: this wave's LDS (and scalar)
// operations complete before it, outstanding global loads may stay in
// flight across it.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Flat grid index of point pt of bigcell o (the index part of point_of).
__device__ inline long long point_index(const GDev &P, const GBig &o, int pt) {
    if (o.w >= 0) return o.w + (((pt >> 4) * P.N[1] + ((pt >> 2) & 3)) * P.N[2] + (pt & 3));
    const int n0 = o.x + (pt >> 4), n1 = o.y + ((pt >> 2) & 3), n2 = o.z + (pt & 3);
    return ((long long)wrapi(n0, P.N[0]) * P.N[1] + wrapi(n1, P.N[1])) * P.N[2] + wrapi(n2, P.N[2]);
}

// Cubic Hermite interpolant on the FP32 table: the interval record of knot k
// ([chan][c0, c1, c2, c3], 16 bytes a channel, the cubic's coefficients in
// t = r/dr - k) and t.
struct Herm32 {
    const float *rec;
    float t, inv_dr;
};

// Knot interval of radius r, found in FP64: with t = r / dr of order 10^3 an
// FP32 t would carry an absolute error of order 1e-4 (a relative error of
// the same order in the interpolation weights); only the offset within the
// interval is rounded to FP32.
struct Knot {
    int k;
    float t;
};

__device__ inline Knot knot_of(CSpecies &sp, double r) {
    const double t = r * sp.inv_dr;
    int k = (int)t;
    if (k > sp.nknots - 2) k = sp.nknots - 2;
    return Knot{k, (float)(t - (double)k)};
}

__device__ __attribute__((always_inline)) inline Herm32 hermite32(CSpecies &sp, const float *tab, Knot kn) {
    Herm32 h;
    h.rec = tab + 2 * (size_t)sp.tab_off + (size_t)kn.k * sp.nchan * 4;
    h.t = kn.t;
    h.inv_dr = (float)sp.inv_dr;
    return h;
}

// p(t) and dp/dt of one channel's record by Horner's rule (no cancellation:
// each term is of the size of the derivative it carries)
__device__ inline float cubic_val(const flt4_t &c, float t) { return fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x); }
__device__ inline float cubic_dt(const flt4_t &c, float t) {
    return fmaf(fmaf(3.f * c.w, t, 2.f * c.z), t, c.y);
}

// Coefficient records of up to RCH32 channels, all loads issued before any
// is used (a loop that loads as it goes waits one memory round trip per
// channel).
constexpr int RCH32 = 5;

struct Rows32 {
    flt4_t c[RCH32];
};

__device__ __attribute__((always_inline)) inline void load_rows32(const Herm32 &h, int nchan, int c0, Rows32 &R) {
#pragma unroll
    for (int q = 0; q < RCH32; ++q)
        if (c0 + q < nchan) R.c[q] = *(const flt4_t *)(h.rec + 4 * (c0 + q));
}

// phi_mu(x) * scale in FP32 for the 16 slots of one atom, handed to emit(mu, v),
// from the Hermite weights h and the already requested first chunk of table
// rows R0 (the caller can issue those loads early).
template <int SHAPE, class Emit>
__device__ __attribute__((always_inline)) inline void eval32_rows(CSpecies &sp, const Herm32 &h, const Rows32 &R0, float x, float y, float z,
                                   float scale, Emit emit) {
    const float S20 = x * y, S21 = y * z, S22 = mulQ(2.f * z * z - x * x - y * y), S23 = x * z,
                S24 = 0.5f * (x * x - y * y);
    const int nchan = ChanShape<SHAPE>::nchan(sp);
    int slot = 0;
    for (int c0 = 0; c0 < nchan; c0 += RCH32) {
        Rows32 R;
        if (c0 == 0)
            R = R0;
        else
            load_rows32(h, nchan, c0, R);
#pragma unroll
        for (int q = 0; q < RCH32; ++q) {
            if (c0 + q >= nchan) break;
            const float p = cubic_val(R.c[q], h.t) * scale;
            const int l = ChanShape<SHAPE>::l(sp, c0 + q);
            if (l == 0) {
                emit(slot, p);
                slot += 1;
            } else if (l == 1) {
                emit(slot, p * y);
                emit(slot + 1, p * z);
                emit(slot + 2, p * x);
                slot += 3;
            } else {
                emit(slot, p * S20);
                emit(slot + 1, p * S21);
                emit(slot + 2, p * S22);
                emit(slot + 3, p * S23);
                emit(slot + 4, p * S24);
                slot += 5;
            }
        }
    }
    for (; slot < GINT_ORB; ++slot) emit(slot, 0.f);
}

template <int SHAPE, class Emit>
__device__ __attribute__((always_inline)) inline void eval32(CSpecies &sp, const float *tab, float x, float y, float z, Knot kn, float scale,
                              Emit emit) {
    const Herm32 h = hermite32(sp, tab, kn);
    Rows32 R0;
    load_rows32(h, ChanShape<SHAPE>::nchan(sp), 0, R0);
    eval32_rows<SHAPE>(sp, h, R0, x, y, z, scale, emit);
}

// sum_mu psi_mu phi_mu and sum_mu psi_mu grad phi_mu, FP32, from the Hermite
// weights and the first chunk of table rows (as eval32_rows).
template <int SHAPE>
__device__ __attribute__((always_inline)) inline void dot_grad32_rows(CSpecies &sp, const Herm32 &h, const Rows32 &R0, float x, float y, float z,
                                       float inv_r, const float *psi, float &e, float G[3]) {
    e = 0.f;
    G[0] = G[1] = G[2] = 0.f;
    const float dscale = h.inv_dr * inv_r;
    const int nchan = ChanShape<SHAPE>::nchan(sp);
    int slot = 0;
    for (int c0 = 0; c0 < nchan; c0 += RCH32) {
      Rows32 R;
      if (c0 == 0)
          R = R0;
      else
          load_rows32(h, nchan, c0, R);
#pragma unroll
      for (int qq = 0; qq < RCH32; ++qq) {
        if (c0 + qq >= nchan) break;
        const float p = cubic_val(R.c[qq], h.t);
        const float q = cubic_dt(R.c[qq], h.t) * dscale;   // p'(r) / r
        const int l = ChanShape<SHAPE>::l(sp, c0 + qq);
        float A, Bx, By, Bz;
        if (l == 0) {
            A = psi[slot];
            Bx = By = Bz = 0.f;
            slot += 1;
        } else if (l == 1) {
            const float p0 = psi[slot], p1 = psi[slot + 1], p2 = psi[slot + 2];
            A = p0 * y + p1 * z + p2 * x;
            Bx = p2;
            By = p0;
            Bz = p1;
            slot += 3;
        } else {
            const float p0 = psi[slot], p1 = psi[slot + 1], p2 = psi[slot + 2], p3 = psi[slot + 3], p4 = psi[slot + 4];
            const float q2 = mulQ(p2), h4 = 0.5f * p4;
            A = p0 * x * y + p1 * y * z + p3 * x * z + q2 * (2.f * z * z - x * x - y * y) + h4 * (x * x - y * y);
            Bx = p0 * y + p3 * z - 2.f * q2 * x + 2.f * h4 * x;
            By = p0 * x + p1 * z - 2.f * q2 * y - 2.f * h4 * y;
            Bz = p1 * y + p3 * x + 4.f * q2 * z;
            slot += 5;
        }
        e += p * A;
        G[0] += q * A * x + p * Bx;
        G[1] += q * A * y + p * By;
        G[2] += q * A * z + p * Bz;
      }
    }
}

template <int SHAPE>
__device__ __attribute__((always_inline)) inline void dot_grad32(CSpecies &sp, const float *tab, float x, float y, float z, Knot kn, float inv_r,
                                  const float *psi, float &e, float G[3]) {
    const Herm32 h = hermite32(sp, tab, kn);
    Rows32 R0;
    load_rows32(h, ChanShape<SHAPE>::nchan(sp), 0, R0);
    dot_grad32_rows<SHAPE>(sp, h, R0, x, y, z, inv_r, psi, e, G);
}

// Activity of one atom at one point; x is the FP32 displacement.
struct Disp {
    float x, y, z;
    Knot kn;
    bool in;
};

// Position (tau + lattice shift) and species of the atom in one slot of the
// current work item, read once per item: the Vlocal bigcell loop then issues
// no dependent atom -> species descriptor loads.  species < 0: empty slot.
struct Slot {
    double x, y, z;
    int species;
};

__device__ inline Slot slot_of(const GDev &P, int atom, cdouble *shift) {
    Slot s{0.0, 0.0, 0.0, -1};
    if (atom >= 0) {
        const GAtom at = ldc(P.atoms + atom);
        s.x = at.x + shift[0];
        s.y = at.y + shift[1];
        s.z = at.z + shift[2];
        s.species = at.species;
    }
    return s;
}

// A slot that is the same in every lane, said so (readfirstlane) so that it
// lives in scalar registers.
__device__ inline double uniform_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b), hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline Slot uniform_slot(const Slot &s) {
    return Slot{uniform_f64(s.x), uniform_f64(s.y), uniform_f64(s.z), __builtin_amdgcn_readfirstlane(s.species)};
}

// The same from the atom index (descriptors loaded at the call; the rho and
// force kernels use this form: holding two slots there costs more registers
// than the loads).
__device__ inline Disp disp_of(const GDev &P, const P3 &r, int atom, cdouble *shift) {
    Disp d{0.f, 0.f, 0.f, Knot{0, 0.f}, false};
    if (atom < 0) return d;
    const GAtom at = ldc(P.atoms + (atom));
    const double dx = r.x - at.x - shift[0], dy = r.y - at.y - shift[1], dz = r.z - at.z - shift[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    CSpecies &sp = cst(P.species)[at.species];
    const double rr = sqrt(r2);
    d.in = r2 < sp.rcut2 && rr < sp.rcut;
    d.x = (float)dx;
    d.y = (float)dy;
    d.z = (float)dz;
    if (d.in) d.kn = knot_of(sp, rr);
    return d;
}

// sqrt(r2) for r2 >= 0 to near FP64 accuracy: the FP32 reciprocal square
// root (relative error about 2e-7 after the conversions) refined by one
// Newton step in FP64, r1 = r0 + (r2 - r0^2) / (2 r0), which squares the
// relative error (about 1e-13).  Five FP64-class operations against about a
// dozen for the correctly rounded square root.  r2 below the FP32 range
// (r < 1e-19) gives 0.
__device__ inline double sqrt_r2(double r2) {
    const float f = (float)r2;
    if (!(f > 0.f)) return 0.0;
    const float y = __builtin_amdgcn_rsqf(f);
    const double r0 = (double)(f * y);
    return fma(fma(-r0, r0, r2), (double)(0.5f * y), r0);
}

__device__ inline Disp disp_at(const GDev &P, const P3 &r, const Slot &s) {
    Disp d{0.f, 0.f, 0.f, Knot{0, 0.f}, false};
    if (s.species < 0) return d;
    const double dx = r.x - s.x, dy = r.y - s.y, dz = r.z - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    CSpecies &sp = cst(P.species)[s.species];
    d.x = (float)dx;
    d.y = (float)dy;
    d.z = (float)dz;
    if (r2 < sp.rcut2) {
        const double rr = sqrt_r2(r2);
        d.in = rr < sp.rcut;
        if (d.in) d.kn = knot_of(sp, rr);
    }
    return d;
}

// A slot with the cutoff and table constants of its species, read once per
// work item, so that a loop over bigcells issues no species descriptor loads.
struct SlotC {
    Slot s;
    double rcut2, rcut, inv_dr;
    int kmax;            // last knot interval
    const float *rec0;   // FP32 table records of the species
};

__device__ inline SlotC slot_consts(const GDev &P, const Slot &s) {
    SlotC c{s, 0.0, 0.0, 0.0, 0, P.tab32};
    if (s.species >= 0) {
        CSpecies &sp = cst(P.species)[s.species];
        c.rcut2 = sp.rcut2;
        c.rcut = sp.rcut;
        c.inv_dr = sp.inv_dr;
        c.kmax = sp.nknots - 2;
        c.rec0 = P.tab32 + 2 * (size_t)sp.tab_off;
    }
    return c;
}

// disp_at with the constants of c (the same arithmetic, knot_of included).
__device__ inline Disp disp_c(const P3 &r, const SlotC &c) {
    Disp d{0.f, 0.f, 0.f, Knot{0, 0.f}, false};
    if (c.s.species < 0) return d;
    const double dx = r.x - c.s.x, dy = r.y - c.s.y, dz = r.z - c.s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    d.x = (float)dx;
    d.y = (float)dy;
    d.z = (float)dz;
    if (r2 < c.rcut2) {
        const double rr = sqrt_r2(r2);
        d.in = rr < c.rcut;
        if (d.in) {
            const double t = rr * c.inv_dr;
            int k = (int)t;
            if (k > c.kmax) k = c.kmax;
            d.kn = Knot{k, (float)(t - (double)k)};
        }
    }
    return d;
}

// Hermite record of knot interval kn of the species of c (as hermite32).
__device__ inline Herm32 hermite_c(const SlotC &c, Knot kn, int nchan) {
    Herm32 h;
    h.rec = c.rec0 + (size_t)kn.k * nchan * 4;
    h.t = kn.t;
    h.inv_dr = (float)c.inv_dr;
    return h;
}

// Whether slot s reaches point r: the r2 part of disp_at's test alone (a
// superset of disp_at's d.in, which also requires sqrt(r2) < rcut; the two
// differ only within an ulp of the cutoff sphere, where the orbitals vanish).
__device__ inline bool reaches(const GDev &P, const P3 &r, const Slot &s) {
    if (s.species < 0) return false;
    const double dx = r.x - s.x, dy = r.y - s.y, dz = r.z - s.z;
    return dx * dx + dy * dy + dz * dz < cst(P.species)[s.species].rcut2;
}

// Orbital rows of a Vlocal tile that reach stored outputs: the orbital
// count of a fixed channel layout, else all 16.
template <int KS>
__device__ constexpr int rows_used() {
    if constexpr (KS == GINT_SHAPE_ANY)
        return 16;
    else
        return ChanShape<KS>::norb;
}

// Whether any lane of this lane's 32-lane half has the flag set (the
// ballot is taken by every lane, so call it where the whole wave is).
__device__ inline bool half_active(bool flag) {
    const unsigned long long b = __ballot(flag);
    return ((b >> (threadIdx.x & 32)) & 0xffffffffull) != 0ull;
}

constexpr int TSTR = 72;   // 16-bit elements per tile row (64 points + 8): conflict-free 16-byte reads

// Power of two s with m s in [2^12, 2^13) (1 if m is 0 or not finite),
// exponent clamped to +-60: operands m s stay below 2^13 and well above the
// FP16 subnormal range, and undoing s is exact.
__device__ inline float pow2_scale(double m) {
    if (!(m > 0.0) || !(m < 1e300)) return 1.f;
    int e;
    (void)frexp(m, &e);
    int k = 13 - e;
    k = k < -60 ? -60 : (k > 60 ? 60 : k);
    return ldexpf(1.f, k);
}

// One (point, slot) row of the B tile for a fixed channel layout: the
// orbital indices are compile-time constants, so the 16 hi and 16 lo values
// are gathered in registers (orbitals arrive in increasing order, so a pair
// completes at each odd index) and written with 16-byte stores.  With
// 144-byte point rows each 16 lanes of such a store hit distinct banks;
// 2-byte stores conflict 4-way.
template <class T, int SH>
__device__ __attribute__((always_inline)) inline void stage_b16_rows(CSpecies &sp, const float *tab, const Disp &d,
                                                                     float sphi, T *h0, T *h1) {
    u4v hv[2], lv[2];
    float pend = 0.f;
    eval32<SH>(sp, tab, d.x, d.y, d.z, d.kn, sphi, [&](int mu, float v) {
        if constexpr (Split16<T>::pairs) {
            if (mu & 1) {
                unsigned h2, l2;
                Split16<T>::split2(pend, v, h2, l2);
                hv[mu >> 3][(mu & 7) >> 1] = h2;
                lv[mu >> 3][(mu & 7) >> 1] = l2;
            } else {
                pend = v;
            }
        } else {
            T hi, lo;
            Split16<T>::split(v, hi, lo);
            const unsigned sh = 16 * (mu & 1);
            const unsigned hb = __builtin_bit_cast(unsigned short, hi), lb = __builtin_bit_cast(unsigned short, lo);
            const int k = mu >> 3, e = (mu & 7) >> 1;
            hv[k][e] = (mu & 1) ? (hv[k][e] | (hb << sh)) : hb;
            lv[k][e] = (mu & 1) ? (lv[k][e] | (lb << sh)) : lb;
        }
    });
    *(u4v *)h0 = hv[0];
    *(u4v *)(h0 + 8) = hv[1];
    *(u4v *)h1 = lv[0];
    *(u4v *)(h1 + 8) = lv[1];
}

}  // namespace
