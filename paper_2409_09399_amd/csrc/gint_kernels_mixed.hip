// Mixed-precision grid integration on CDNA4 (gfx950).
//
// Same work decomposition as the FP64 kernels (cluster-pair items over
// 4x4x4-point bigcells, see gint_internal.h), different arithmetic:
//   - orbitals are evaluated in FP32 from FP32 radial tables;
//   - every MFMA operand x is split into 16-bit parts x = x_hi + x_lo
//     (FP16 or BF16) and a product is a_hi b_hi + a_hi b_lo + a_lo b_hi on
//     v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation (the dropped
//     a_lo b_lo term is below the split's own rounding);
//   - FP32 partial sums of one bigcell are folded into FP64 accumulators,
//     and H, rho, F, Z, E and N_e are reduced in FP64.
// The local potential enters the Vlocal operand as V (not w V) so that the
// 16-bit parts stay in range; the constant w is applied in FP64.
#include <hip/hip_runtime.h>

#include "gint_mixed.h"

// ---------------------------------------------------------------------------
// H_IJR (Eq. 2), mixed precision.  Tiles [A/B][hi/lo][slot][orbital][point].
// Eight waves, one orbital set each per bigcell: wave w < 4 evaluates A atom
// w, wave w >= 4 the V-weighted B atom w - 4, so a wave waits for one table
// (and V) round trip per bigcell.  In the contraction wave w owns the two
// tiles (a_i, b_j) with i = w & 3 and j = i + 2 (w >> 2) + {0, 1} (mod 4):
// every slot's tiles spread over two waves, and one A fragment read serves
// both products.  Two k-steps of 32 points.  A pass over a bigcell is a
// latency chain (table round trip, evaluation, barrier, MFMA, fold), so the
// kernel is held to 80 registers: three workgroups per CU (six waves per SIMD).
// Its barriers order LDS only, so the V of the next bigcell, requested after
// this one's table loads, stays in flight across them.  The slot's species
// constants (cutoffs, knot spacing, table base) are read once per item, so a
// bigcell's chain holds no scalar descriptor round trips beyond its own.
// ---------------------------------------------------------------------------
template <class T, int KS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_vlocal_mx(GDev P0, const double *__restrict__ V0, double *__restrict__ H) {
    typedef Split16<T> S;
    typedef typename S::vec vec;
    __shared__ __attribute__((aligned(16))) T tS[2][2][4][16][TSTR];
    // per wave and bigcell: bit kk set if its atom reaches a point of k-step kk
    __shared__ __attribute__((aligned(16))) unsigned s_act[8];
    __shared__ int s_item;
    // A = phi * sphi, B = V phi * sB, both below 2^13 in magnitude
    const float sphi = (float)P0.phi_scale;
    const float sB = pow2_scale(*cst(P0.vmax) * (8192.0 / P0.phi_scale));
    const double unscale = 1.0 / ((double)sphi * (double)sB);
    const int lane = threadIdx.x & 63, w = wave_id();
    const int set = w >> 2, slot = w & 3;
    for (;;) {
    const int item_ = claim_item(P0.counter, &s_item);
    if (item_ >= P0.nitems) break;
    const GItem it = ldc(P0.items + item_);
    CPair &pr = cst(P0.pairs)[it.pair];
    GDev P = P0;
    bind_system(P, pr.sys);
    CSys &SY = cst(P0.sys)[pr.sys];
    const double *V = V0 + SY.g_off;
    const Slot sl = uniform_slot(set ? slot_of(P, pr.b[slot], pr.shiftB) : slot_of(P, pr.a[slot], pr.shiftA));
    const SlotC slc = slot_consts(P, sl);
    const int i = slot, j0 = (slot + 2 * set) & 3, j1 = (j0 + 1) & 3;
    d4v acc[2];
    acc[0] = acc[1] = (d4v){0.0, 0.0, 0.0, 0.0};

    const int pt = lane;
    // FP16 tiles of a fixed orbital layout are stored 32 bits at a time:
    // lanes 2k and 2k + 1 exchange their converted pairs of rows, and the
    // even lane stores the lower row at points 2k, 2k + 1, the odd lane the
    // upper (half the stores of 16-bit ones, and no two lanes in one bank
    // word).  poff: this lane's byte offset within a pair of rows; psel: the
    // byte selector that takes its half from each lane's pair.
    constexpr bool PACK = S::pairs && KS != GINT_SHAPE_ANY;
    const int poff = (lane & 1) * (TSTR * 2) + (lane & ~1) * 2;
    const unsigned psel = (lane & 1) ? 0x03020706u : 0x05040100u;
    // V of the first bigcell; the next one's is requested after each
    // bigcell's table loads (so they are not waited for together) and stays
    // in flight across the LDS-only barriers
    double vn = set ? V[point_index(P, ldc(P.bigcells + it.bc_begin), pt)] : 0.0;
    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        {
            // phase 1: this wave's atom at point lane
            const P3 r = point_of(P, o, pt);
            const float vpt = (float)vn;
            const Disp d = disp_c(r, slc);
            const unsigned long long bl = __ballot(d.in);
            const bool zero = ((bl >> (lane & 32)) & 0xffffffffull) != 0ull;
            // with paired stores both lanes of a pair evaluate when either
            // is active, the inactive one with weight 0
            const bool ev = PACK ? ((bl >> (lane & ~1)) & 3ull) != 0ull : d.in;
            if (ev) {
                CSpecies &sp = cst(P.species)[sl.species];
                const float sc = d.in ? (set ? vpt * sB : sphi) : 0.f;
                float pend = 0.f;
                with_shape<KS>(sp, [&](auto shp) {
                    constexpr int SH = decltype(shp)::value;
                    const Herm32 hm = hermite_c(slc, d.kn, ChanShape<SH>::nchan(sp));
                    Rows32 R0;
                    load_rows32(hm, ChanShape<SH>::nchan(sp), 0, R0);
                    eval32_rows<SH>(sp, hm, R0, d.x, d.y, d.z, sc, [&](int mu, float v) {
                        T hi, lo;
                        if constexpr (SH != GINT_SHAPE_ANY) {
                            // padding rows reach only output rows or columns
                            // beyond the orbital count, which are never stored
                            constexpr int NO = ChanShape<SH>::norb;
                            if (mu >= NO) return;
                            if constexpr (S::pairs) {
                                // orbitals arrive in increasing order: convert
                                // them two at a time, each half stored to its row
                                if (!(mu & 1) && mu + 1 < NO) {
                                    pend = v;
                                    return;
                                }
                                if (mu & 1) {
                                    unsigned h2, l2;
                                    S::split2(pend, v, h2, l2);
                                    if constexpr (PACK) {
                                        // the partner lane's pairs (quad_perm [1,0,3,2]; every
                                        // lane is active, so no old value is needed)
                                        const unsigned oh = __builtin_amdgcn_mov_dpp(h2, 0xB1, 0xF, 0xF, true);
                                        const unsigned ol = __builtin_amdgcn_mov_dpp(l2, 0xB1, 0xF, 0xF, true);
                                        *(unsigned *)((char *)&tS[set][0][slot][mu - 1][0] + poff) = __builtin_amdgcn_perm(oh, h2, psel);
                                        *(unsigned *)((char *)&tS[set][1][slot][mu - 1][0] + poff) = __builtin_amdgcn_perm(ol, l2, psel);
                                    } else {
                                        *(unsigned short *)&tS[set][0][slot][mu - 1][pt] = (unsigned short)h2;
                                        *(unsigned short *)&tS[set][0][slot][mu][pt] = (unsigned short)(h2 >> 16);
                                        *(unsigned short *)&tS[set][1][slot][mu - 1][pt] = (unsigned short)l2;
                                        *(unsigned short *)&tS[set][1][slot][mu][pt] = (unsigned short)(l2 >> 16);
                                    }
                                    return;
                                }
                            }
                            S::split_mix(v, hi, lo);
                        } else {
                            S::split(v, hi, lo);
                        }
                        tS[set][0][slot][mu][pt] = hi;
                        tS[set][1][slot][mu][pt] = lo;
                    });
                });
            } else if (zero) {
                // zeros only where the half is read: a 32-point k-step of
                // this slot's tile enters the products only if the atom is
                // active somewhere in it
                if constexpr (PACK) {
                    // both lanes of a pair are here
                    constexpr int NO = rows_used<KS>();
#pragma unroll
                    for (int mu = 1; mu < NO; mu += 2) {
                        *(unsigned *)((char *)&tS[set][0][slot][mu - 1][0] + poff) = 0u;
                        *(unsigned *)((char *)&tS[set][1][slot][mu - 1][0] + poff) = 0u;
                    }
                    if constexpr (NO & 1) {
                        tS[set][0][slot][NO - 1][pt] = (T)0.f;
                        tS[set][1][slot][NO - 1][pt] = (T)0.f;
                    }
                } else {
#pragma unroll
                    for (int mu = 0; mu < rows_used<KS>(); ++mu) {
                        tS[set][0][slot][mu][pt] = (T)0.f;
                        tS[set][1][slot][mu][pt] = (T)0.f;
                    }
                }
            }
            if (lane == 0) s_act[w] = ((unsigned)bl != 0u ? 1u : 0u) | ((unsigned)(bl >> 32) != 0u ? 2u : 0u);
            if (set && bc + 1 < it.bc_count) vn = V[point_index(P, ldc(P.bigcells + it.bc_begin + bc + 1), pt)];
        }
        lds_barrier();
        // phase 2: the two tiles of this wave
        const unsigned actA = s_act[i], actB0 = s_act[4 + j0], actB1 = s_act[4 + j1];
        f4v c0 = (f4v){0.f, 0.f, 0.f, 0.f}, c1 = (f4v){0.f, 0.f, 0.f, 0.f};
        const int row = lane & 15, col = 8 * (lane >> 4);
        bool any0 = false, any1 = false;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const bool b0 = ((actA & actB0) >> kk) & 1u, b1 = ((actA & actB1) >> kk) & 1u;
            if (!b0 && !b1) continue;
            const vec ahi = *(const vec *)&tS[0][0][i][row][32 * kk + col];
            const vec alo = *(const vec *)&tS[0][1][i][row][32 * kk + col];
            if (b0) {
                const vec bhi = *(const vec *)&tS[1][0][j0][row][32 * kk + col];
                const vec blo = *(const vec *)&tS[1][1][j0][row][32 * kk + col];
                c0 = S::mfma(ahi, bhi, c0);
                c0 = S::mfma(ahi, blo, c0);
                c0 = S::mfma(alo, bhi, c0);
                any0 = true;
            }
            if (b1) {
                const vec bhi = *(const vec *)&tS[1][0][j1][row][32 * kk + col];
                const vec blo = *(const vec *)&tS[1][1][j1][row][32 * kk + col];
                c1 = S::mfma(ahi, bhi, c1);
                c1 = S::mfma(ahi, blo, c1);
                c1 = S::mfma(alo, bhi, c1);
                any1 = true;
            }
        }
        // the tiles are free once this wave's fragment reads have returned:
        // the products are folded into FP64 after the barrier
        lds_barrier();
        if (any0)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[0][q] += (double)c0[q];
        if (any1)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[1][q] += (double)c1[q];
    }
    // 16x16x32 result layout: lane l, register q holds row 4 (l >> 4) + q, column l & 15
    const bool exclusive = it.pad != 0;
    const int nu = lane & 15;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int j = t ? j1 : j0;
        const int ai = pr.a[i], bj = pr.b[j];
        if (ai < 0 || bj < 0) continue;
        const int na = cst(P.atoms)[ai].norb, nb = cst(P.atoms)[bj].norb;
        const long long off = pr.hoff[i * 4 + j], offt = pr.hoff_t[i * 4 + j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int mu = 4 * (lane >> 4) + q;
            if (mu >= na || nu >= nb) continue;
            const double v = P.w * unscale * acc[t][q];
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

// ---------------------------------------------------------------------------
// H_IJR (Eq. 2), mixed precision, clusters of up to eight atoms.  Eight
// waves: wave w evaluates A atom w and B atom w on the bigcell's 64 points
// (one point per lane) and owns the eight tiles (a_i, b_{(w-i)&7}); two
// k-steps of 32 points.  Against the four-atom kernel every evaluation feeds
// twice the tiles, which is what bounds this stage: per bigcell it is VALU
// (orbital evaluation), not MFMA, work.  The FP32 tiles of a bigcell are
// formed four at a time and folded into FP64 accumulators.
// ---------------------------------------------------------------------------
template <class T, int KS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_vlocal_mx8(
    GDev P0, const double *__restrict__ V0, double *__restrict__ H) {
    typedef Split16<T> S;
    typedef typename S::vec vec;
    __shared__ __attribute__((aligned(16))) T tA[2][GINT_CL8][16][TSTR];
    __shared__ __attribute__((aligned(16))) T tB[2][GINT_CL8][16][TSTR];
    __shared__ unsigned maskpt2[2][GINT_BCPTS];
    __shared__ int s_item;
    const float sphi = (float)P0.phi_scale;
    const float sB = pow2_scale(*cst(P0.vmax) * (8192.0 / P0.phi_scale));
    const double unscale = 1.0 / ((double)sphi * (double)sB);
    // double-buffered activity mask (bits 0-7: A slots, 8-15: B slots)
    if (threadIdx.x < 2 * GINT_BCPTS) maskpt2[threadIdx.x >> 6][threadIdx.x & 63] = 0u;
    int cur = 0;
    for (;;) {
    const int item_ = claim_item(P0.counter, &s_item);
    if (item_ >= P0.nitems) break;
    const GItem it = ldc(P0.items + item_);
    CPair8 &pr = cst(P0.pairs8)[it.pair];
    GDev P = P0;
    bind_system(P, pr.sys);
    CSys &SY = cst(P0.sys)[pr.sys];
    const double *V = V0 + SY.g_off;
    const int lane = threadIdx.x & 63, w = wave_id();
    const Slot sa = slot_of(P, pr.a[w], pr.shiftA), sb = slot_of(P, pr.b[w], pr.shiftB);
    d4v acc[GINT_CL8];
#pragma unroll
    for (int i = 0; i < GINT_CL8; ++i) acc[i] = (d4v){0.0, 0.0, 0.0, 0.0};

    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        unsigned *maskpt = maskpt2[cur];
        {
            const int pt = lane;
            const P3 r = point_of(P, o, pt);
            const double vpt = V[r.g];
            unsigned bits = 0;
            const Disp da = disp_at(P, r, sa);
            const bool zA = half_active(da.in);
            if (da.in) {
                CSpecies &sp = cst(P.species)[sa.species];
                with_shape<KS>(sp, [&](auto shp) {
                    eval32<decltype(shp)::value>(sp, P.tab32, da.x, da.y, da.z, da.kn, sphi, [&](int mu, float v) {
                        T hi, lo;
                        constexpr int SH = decltype(shp)::value;
                        if constexpr (SH != GINT_SHAPE_ANY) {
                            if (mu >= ChanShape<SH>::norb) return;
                            S::split_mix(v, hi, lo);
                        } else {
                            S::split(v, hi, lo);
                        }
                        tA[0][w][mu][pt] = hi;
                        tA[1][w][mu][pt] = lo;
                    });
                });
                bits |= 1u << w;
            } else if (zA) {
#pragma unroll
                for (int mu = 0; mu < rows_used<KS>(); ++mu) {
                    tA[0][w][mu][pt] = (T)0.f;
                    tA[1][w][mu][pt] = (T)0.f;
                }
            }
            const Disp db = disp_at(P, r, sb);
            const bool zB = half_active(db.in);
            if (db.in) {
                CSpecies &sp = cst(P.species)[sb.species];
                const float vg = (float)vpt * sB;
                with_shape<KS>(sp, [&](auto shp) {
                    eval32<decltype(shp)::value>(sp, P.tab32, db.x, db.y, db.z, db.kn, vg, [&](int mu, float v) {
                        T hi, lo;
                        constexpr int SH = decltype(shp)::value;
                        if constexpr (SH != GINT_SHAPE_ANY) {
                            if (mu >= ChanShape<SH>::norb) return;
                            S::split_mix(v, hi, lo);
                        } else {
                            S::split(v, hi, lo);
                        }
                        tB[0][w][mu][pt] = hi;
                        tB[1][w][mu][pt] = lo;
                    });
                });
                bits |= 1u << (GINT_CL8 + w);
            } else if (zB) {
#pragma unroll
                for (int mu = 0; mu < rows_used<KS>(); ++mu) {
                    tB[0][w][mu][pt] = (T)0.f;
                    tB[1][w][mu][pt] = (T)0.f;
                }
            }
            if (bits) atomicOr(&maskpt[pt], bits);
        }
        __syncthreads();
        if (threadIdx.x < GINT_BCPTS) maskpt2[cur ^ 1][threadIdx.x] = 0u;
        cur ^= 1;
        // activity of the two 32-point k-steps per slot
        const unsigned mp = maskpt[lane];
        unsigned km[2] = {0u, 0u};
#pragma unroll
        for (int b = 0; b < 2 * GINT_CL8; ++b) {
            const unsigned long long bl = __ballot((mp >> b) & 1u);
            if (bl & 0xffffffffull) km[0] |= 1u << b;
            if (bl >> 32) km[1] |= 1u << b;
        }
        const int row = lane & 15, col = 8 * (lane >> 4);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f4v c32[4];
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) c32[ii] = (f4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
                const int i = 4 * h + ii, j = (w - i) & (GINT_CL8 - 1);
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) {
                    if (!((km[kk] >> i) & 1u) || !((km[kk] >> (GINT_CL8 + j)) & 1u)) continue;
                    const vec ahi = *(const vec *)&tA[0][i][row][32 * kk + col];
                    const vec alo = *(const vec *)&tA[1][i][row][32 * kk + col];
                    const vec bhi = *(const vec *)&tB[0][j][row][32 * kk + col];
                    const vec blo = *(const vec *)&tB[1][j][row][32 * kk + col];
                    c32[ii] = S::mfma(ahi, bhi, c32[ii]);
                    c32[ii] = S::mfma(ahi, blo, c32[ii]);
                    c32[ii] = S::mfma(alo, bhi, c32[ii]);
                }
            }
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[4 * h + ii][q] += (double)c32[ii][q];
        }
        __syncthreads();
    }
    // 16x16x32 result layout: lane l, register q holds row 4 (l >> 4) + q, column l & 15
    const bool exclusive = it.pad != 0;
    const int nu = lane & 15;
#pragma unroll
    for (int i = 0; i < GINT_CL8; ++i) {
        const int j = (w - i) & (GINT_CL8 - 1);
        const int ai = pr.a[i], bj = pr.b[j];
        if (ai < 0 || bj < 0) continue;
        const int na = cst(P.atoms)[ai].norb, nb = cst(P.atoms)[bj].norb;
        const long long off = pr.hoff[i * GINT_CL8 + j], offt = pr.hoff_t[i * GINT_CL8 + j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int mu = 4 * (lane >> 4) + q;
            if (mu >= na || nu >= nb) continue;
            const double v = P.w * unscale * acc[i][q];
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

namespace {

// Row atom i of D_sym as 16-bit hi/lo MFMA B operands for psi = phi_B D^T:
// k-step kk covers B atoms 2kk, 2kk+1; lane l holds mu = l & 15 and
// nu' = 8 (l >> 4) + e, i.e. atom 2kk + (l >> 5), orbital 8 ((l >> 4) & 1) + e.
// The row is scaled by a power of two (its largest entry maps below 2^13);
// returns the factor that undoes the scales of phi and D in psi.
template <class T>
__device__ inline float load_dsym16_row(const GDev &P, CPair &pr, const double *__restrict__ D, int i, float sphi,
                                        typename Split16<T>::vec dh[2], typename Split16<T>::vec dl[2]) {
    const int lane = threadIdx.x & 63;
    const int mu = lane & 15;
    const int na = pr.a[i] >= 0 ? cst(P.atoms)[pr.a[i]].norb : 0;
    float val[2][8];
    float m = 0.f;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const int j = 2 * kk + (lane >> 5);
        const long long o = pr.hoff[i * 4 + j], ot = pr.hoff_t[i * 4 + j];
        const int nb = pr.b[j] >= 0 ? cst(P.atoms)[pr.b[j]].norb : 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int nu = 8 * ((lane >> 4) & 1) + e;
            float v = 0.f;
            if (o >= 0 && ot >= 0 && mu < na && nu < nb)
                v = (float)(0.5 * (D[o + (long long)mu * nb + nu] + D[ot + (long long)nu * na + mu]));
            val[kk][e] = v;
            m = fmaxf(m, fabsf(v));
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    const float sD = pow2_scale((double)m);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            T hi, lo;
            Split16<T>::split(val[kk][e] * sD, hi, lo);
            dh[kk][e] = hi;
            dl[kk][e] = lo;
        }
    return 1.f / (sphi * sD);   // psi = (phi sphi)(D sD) / (sphi sD), exact
}

constexpr int RSTR = 72;   // 16-bit elements per point row of the B tile (4 slots x 16 + 8)
constexpr int FSTR = 65;   // floats per point row of the FP32 psi tile

// Phase 1 of rho/force: B orbitals (scaled by sphi) as 16-bit hi/lo rows
// [h][point][slot*16+mu]; A atoms only mark where they are active.  Returns
// the displacement of A atom a_w from this lane's point r, which the
// per-point phase reuses.
template <class T, int KS>
__device__ inline Disp stage_b16(const GDev &P, CPair &pr, const P3 &r, float sphi, T (*tB)[GINT_BCPTS][RSTR],
                                 unsigned *maskpt, unsigned *maskt) {
    const int lane = threadIdx.x & 63, w = wave_id();
    const int pt = lane;
    unsigned bits = 0;
    const int a = pr.a[w], b = pr.b[w];
    const Disp da = disp_of(P, r, a, pr.shiftA);
    if (da.in) bits |= 1u << w;
    const Disp db = disp_of(P, r, b, pr.shiftB);
    T *h0 = &tB[0][pt][w * 16];
    T *h1 = &tB[1][pt][w * 16];
    if (db.in) {
        CSpecies &sp = cst(P.species)[cst(P.atoms)[b].species];
        with_shape<KS>(sp, [&](auto shp) {
            constexpr int SH = decltype(shp)::value;
            if constexpr (SH != GINT_SHAPE_ANY) {
                stage_b16_rows<T, SH>(sp, P.tab32, db, sphi, h0, h1);
            } else {
                eval32<SH>(sp, P.tab32, db.x, db.y, db.z, db.kn, sphi, [&](int mu, float v) {
                    T hi, lo;
                    Split16<T>::split(v, hi, lo);
                    h0[mu] = hi;
                    h1[mu] = lo;
                });
            }
        });
        bits |= 1u << (4 + w);
    } else {
        const u4v z = {0u, 0u, 0u, 0u};
        *(u4v *)h0 = z;
        *(u4v *)(h0 + 8) = z;
        *(u4v *)h1 = z;
        *(u4v *)(h1 + 8) = z;
    }
    if (bits) atomicOr(&maskpt[pt], bits);
    // activity per 16-point tile, packed in one word (tile t: bit 8t + slot for
    // A, 8t + 4 + slot for B) from the wave's ballots: one atomic per wave
    const unsigned long long ba = __ballot(da.in), bb = __ballot(db.in);
    unsigned tw = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if ((ba >> (16 * t)) & 0xFFFFull) tw |= 1u << (8 * t + w);
        if ((bb >> (16 * t)) & 0xFFFFull) tw |= 1u << (8 * t + 4 + w);
    }
    if (lane == 0 && tw) atomicOr(maskt, tw);
    return da;
}

// Phase 2: wave w computes psi[pt][mu] = sum_{b, nu} phi_B[pt][b nu]
// D_sym[a_w mu][b nu] for the 64 points (four 16-point tiles; tiles where a_w
// is inactive and B-atom pairs inactive on a tile are skipped).  MFMA layout:
// c[t] lane l register q holds point 16 t + 4 (l >> 4) + q, orbital l & 15.
template <class T>
__device__ inline void psi_row16(const typename Split16<T>::vec dh[2], const typename Split16<T>::vec dl[2],
                                 T (*tB)[GINT_BCPTS][RSTR], const unsigned *maskt, f4v c[4]) {
    typedef typename Split16<T>::vec vec;
    const int lane = threadIdx.x & 63, w = wave_id();
    const int off = 8 * (lane >> 4);
    const unsigned all = __builtin_amdgcn_readfirstlane(*maskt);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        c[t] = (f4v){0.f, 0.f, 0.f, 0.f};
        const unsigned gm = (all >> (8 * t)) & 0xFFu;
        if (!(gm & (1u << w))) continue;
        const int pt = 16 * t + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            if (!(gm & (3u << (4 + 2 * kk)))) continue;
            const vec ah = *(const vec *)&tB[0][pt][32 * kk + off];
            const vec al = *(const vec *)&tB[1][pt][32 * kk + off];
            c[t] = Split16<T>::mfma(ah, dh[kk], c[t]);
            c[t] = Split16<T>::mfma(ah, dl[kk], c[t]);
            c[t] = Split16<T>::mfma(al, dh[kk], c[t]);
        }
    }
}

// psi of slot w into its columns of the FP32 tile (after every wave has read tB).
__device__ inline void store_psi32(const f4v c[4], float *psi, const unsigned *maskt, float unscale) {
    const int lane = threadIdx.x & 63, w = wave_id();
    const unsigned all = __builtin_amdgcn_readfirstlane(*maskt);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const unsigned gm = (all >> (8 * t)) & 0xFFu;
        if (!(gm & (1u << w))) continue;
        float *dst = psi + (16 * t + 4 * (lane >> 4)) * FSTR + w * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q * FSTR] = c[t][q] * unscale;
    }
}

// LDS of the rho/force kernels: the B tile, reused for psi after phase 2.
template <class T>
struct TileBuf {
    static constexpr int bytes = 2 * GINT_BCPTS * RSTR * (int)sizeof(T);
    static_assert(bytes >= GINT_BCPTS * FSTR * (int)sizeof(float), "psi must fit in the B tile");
};

}  // namespace

// ---------------------------------------------------------------------------
// rho_g (Eq. 3), mixed precision: canonical pairs, weight 2 off the self
// pair.  Wave w owns A atom slot w: psi by MFMA, then per point (lane)
// phi_{a_w} . psi with phi evaluated on the fly.  The psi tile reuses the B
// tile's LDS (19 KB a workgroup), so six workgroups fit a CU; the fixed-layout
// instance is built for six and the per-species one for five (a few
// registers spill in each, still faster than one workgroup fewer).
// ---------------------------------------------------------------------------
template <class T, int KS>
__global__ __launch_bounds__(256, KS == GINT_SHAPE_ANY ? 5 : 6) void k_rho_mx(GDev P0, const double *__restrict__ D, double *__restrict__ rho0) {
    typedef typename Split16<T>::vec vec;
    __shared__ __attribute__((aligned(16))) unsigned char buf[TileBuf<T>::bytes];
    __shared__ unsigned maskpt[2][GINT_BCPTS];
    __shared__ unsigned maskt[2];
    __shared__ int s_item;
    T(*tB)[GINT_BCPTS][RSTR] = reinterpret_cast<T(*)[GINT_BCPTS][RSTR]>(buf);
    float *psi = reinterpret_cast<float *>(buf);
    const float sphi = (float)P0.phi_scale;
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
    vec dh[2], dl[2];
    const float unscale = load_dsym16_row<T>(P, pr, D, w, sphi, dh, dl);
    const double weight = pr.self ? 1.0 : 2.0;
    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        unsigned *mpt = maskpt[cur], *mt = &maskt[cur];
        const P3 r = point_of(P, o, lane);
        const Disp da = stage_b16<T, KS>(P, pr, r, sphi, tB, mpt, mt);
        __syncthreads();
        // the other buffer was last read before the previous bigcell's final barrier
        if (threadIdx.x < GINT_BCPTS) maskpt[cur ^ 1][threadIdx.x] = 0u;
        if (threadIdx.x == GINT_BCPTS) maskt[cur ^ 1] = 0u;
        cur ^= 1;
        f4v c[4];
        psi_row16<T>(dh, dl, tB, mt, c);
        __syncthreads();
        store_psi32(c, psi, mt, unscale);
        {
            float v = 0.f;
            if (da.in && (mpt[lane] & 0xF0u)) {
                const float *ps = psi + lane * FSTR + w * 16;
                CSpecies &sp = cst(P.species)[cst(P.atoms)[aw].species];
                with_shape<KS>(sp, [&](auto shp) {
                    constexpr int SH = decltype(shp)::value;
                    eval32<SH>(sp, P.tab32, da.x, da.y, da.z, da.kn, 1.f, [&](int mu, float x) {
                        // padding orbitals are zero: no psi read for them
                        if constexpr (SH != GINT_SHAPE_ANY)
                            if (mu >= ChanShape<SH>::norb) return;
                        v += x * ps[mu];
                    });
                });
                // each wave adds its atom's term: no LDS sum over the waves and
                // no barrier for it, at the price of more (FP64) atomics
                atomicAdd(rho + r.g, weight * (double)v);
            }
        }
        __syncthreads();
    }
    }
}

// ---------------------------------------------------------------------------
// Pulay force and strain derivative (Eq. 4-5), mixed precision: ordered
// pairs, A side; FP32 per-point terms, FP64 accumulation.  With RHO the
// per-point values phi_A . psi_A are also added into rho (see k_force).
// ---------------------------------------------------------------------------
template <class T, bool RHO, int KS>
__global__ __launch_bounds__(256, 4) void k_force_mx(GDev P0, const double *__restrict__ V0,
                                                     const double *__restrict__ D, double *__restrict__ F,
                                                     double *__restrict__ ZE0, double *__restrict__ rho0) {
    typedef typename Split16<T>::vec vec;
    __shared__ __attribute__((aligned(16))) unsigned char buf[TileBuf<T>::bytes];
    __shared__ unsigned maskpt[2][GINT_BCPTS];
    __shared__ unsigned maskt[2];
    __shared__ double red[4][10];
    // psi has LDS of its own here (each wave writes and reads only its own
    // columns), so no barrier separates the psi products from the stores; at
    // four workgroups per CU (the register limit) the extra LDS costs no occupancy
    __shared__ float psi[GINT_BCPTS * FSTR];
    __shared__ int s_item;
    T(*tB)[GINT_BCPTS][RSTR] = reinterpret_cast<T(*)[GINT_BCPTS][RSTR]>(buf);
    const float sphi = (float)P0.phi_scale;
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
    vec dh[2], dl[2];
    const float unscale = load_dsym16_row<T>(P, pr, D, w, sphi, dh, dl);
    double f[3] = {0, 0, 0}, z[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, en = 0.0;
    for (int bc = 0; bc < it.bc_count; ++bc) {
        const GBig o = ldc(P.bigcells + it.bc_begin + bc);
        unsigned *mpt = maskpt[cur], *mt = &maskt[cur];
        const P3 r = point_of(P, o, lane);
        const double vpt = V[r.g];   // requested early: its latency overlaps the stage
        const Disp da = stage_b16<T, KS>(P, pr, r, sphi, tB, mpt, mt);
        __syncthreads();
        // the other buffer was last read before the previous bigcell's final barrier
        if (threadIdx.x < GINT_BCPTS) maskpt[cur ^ 1][threadIdx.x] = 0u;
        if (threadIdx.x == GINT_BCPTS) maskt[cur ^ 1] = 0u;
        cur ^= 1;
        f4v c[4];
        psi_row16<T>(dh, dl, tB, mt, c);
        store_psi32(c, psi, mt, unscale);
        double ev = 0.0;
        if (da.in && (mpt[lane] & 0xF0u)) {
            CSpecies &sp = cst(P.species)[ldc(P.atoms + aw).species];
            // |r - tau| from the knot: (k + t) dr, relative error ~1e-7
            const float rr = ((float)da.kn.k + da.kn.t) * (float)sp.dr;
            float e, G[3];
            with_shape<KS>(sp, [&](auto shp) {
                dot_grad32<decltype(shp)::value>(sp, P.tab32, da.x, da.y, da.z, da.kn, rr > 0.f ? __builtin_amdgcn_rcpf(rr) : 0.f,
                                                 psi + lane * FSTR + w * 16, e, G);
            });
            const double wv = P.w * vpt;
            const double c2 = 2.0 * wv;
            const double g0 = G[0], g1 = G[1], g2 = G[2];
            f[0] += c2 * g0;
            f[1] += c2 * g1;
            f[2] += c2 * g2;
            const double gs[3] = {g0, g1, g2}, xs[3] = {da.x, da.y, da.z};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) z[3 * a + b] += c2 * gs[a] * xs[b];
            en += wv * (double)e;
            ev = (double)e;
        }
        // each wave adds its atom's rho term (over the two orders of a pair this
        // gives rho's weight 2 off the self pair)
        if (RHO && ev != 0.0) atomicAdd(rho + r.g, ev);
        __syncthreads();
    }
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
// launchers
// ---------------------------------------------------------------------------
int gint_persistent_grid(const void *kernel, int nitems, int threads);
hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s);


// max |x| into *out (non-negative doubles order like their bit patterns)
__global__ __launch_bounds__(256) void k_absmax(const double *__restrict__ x, long long n,
                                                unsigned long long *__restrict__ out) {
    double m = 0.0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) m = fmax(m, fabs(x[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// max |x| over n doubles into *out (which the caller has cleared)
hipError_t gint_launch_absmax(const double *x, long long n, double *out, hipStream_t s) {
    long long blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, s, x, n, (unsigned long long *)out);
    return hipGetLastError();
}

// Kernel instances per (16-bit type, plan-wide species layout): plans whose
// species are all 2s2p1d run the instance with that layout fixed, others the
// one that branches per species.
struct KVlocal {
    template <class T, int KS>
    static const void *get() { return (const void *)k_vlocal_mx<T, KS>; }
};
struct KVlocal8 {
    template <class T, int KS>
    static const void *get() { return (const void *)k_vlocal_mx8<T, KS>; }
};
struct KRho {
    template <class T, int KS>
    static const void *get() { return (const void *)k_rho_mx<T, KS>; }
};
template <bool RHO>
struct KForce {
    template <class T, int KS>
    static const void *get() { return (const void *)k_force_mx<T, RHO, KS>; }
};

template <class K>
const void *kernel_for(int prec, int shape_all) {
    const bool fixed = shape_all == GINT_SHAPE_2S2P1D;
    if (prec == 2)
        return fixed ? K::template get<__bf16, GINT_SHAPE_2S2P1D>() : K::template get<__bf16, GINT_SHAPE_ANY>();
    return fixed ? K::template get<_Float16, GINT_SHAPE_2S2P1D>() : K::template get<_Float16, GINT_SHAPE_ANY>();
}

template <class K, int THREADS = 256, class... Args>
hipError_t launch_form(const GDev &P, int prec, hipStream_t s, Args... args) {
    const void *k = kernel_for<K>(prec, P.shape_all);
    if (P.nitems <= 0) return hipSuccess;
    hipError_t e = gint_launch_fill((double *)P.counter, 1, 0.0, s);
    if (e != hipSuccess) return e;
    const int grid = gint_persistent_grid(k, P.nitems, THREADS);
    void *argv[] = {const_cast<GDev *>(&P), &args...};
    e = hipLaunchKernel(k, dim3(grid), dim3(THREADS), argv, 0, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// max |V| over the ngrid points of V into P.vmax, from which the mixed
// Vlocal kernels take the scale of their B operand
hipError_t gint_launch_vmax(const GDev &P, const double *V, long long ngrid, hipStream_t s) {
    hipError_t e = gint_launch_fill(const_cast<double *>(P.vmax), 1, 0.0, s);
    if (e != hipSuccess) return e;
    return gint_launch_absmax(V, ngrid, const_cast<double *>(P.vmax), s);
}

// the mixed Vlocal kernel alone (P.vmax already holds max |V| of this V)
hipError_t gint_launch_vlocal_mx_prepared(const GDev &P, int prec, const double *V, double *H, hipStream_t s) {
    if (P.pairs8) return launch_form<KVlocal8, 512>(P, prec, s, V, H);
    return launch_form<KVlocal, 512>(P, prec, s, V, H);
}

hipError_t gint_launch_vlocal_mx(const GDev &P, int prec, const double *V, long long ngrid, double *H,
                                 hipStream_t s) {
    hipError_t e = gint_launch_vmax(P, V, ngrid, s);
    if (e != hipSuccess) return e;
    return gint_launch_vlocal_mx_prepared(P, prec, V, H, s);
}

hipError_t gint_launch_rho_mx(const GDev &P, int prec, const double *D, double *rho, hipStream_t s) {
    return launch_form<KRho>(P, prec, s, D, rho);
}

hipError_t gint_launch_force_mx(const GDev &P, int prec, const double *V, const double *D, double *F, double *ZE,
                                double *rho, hipStream_t s) {
    if (rho) return launch_form<KForce<true>>(P, prec, s, V, D, F, ZE, rho);
    return launch_form<KForce<false>>(P, prec, s, V, D, F, ZE, (double *)nullptr);
}

int gint_resident_blocks(const void *kernel, int threads);

void gint_prime_grids_mx(int prec) {
    for (int shape : {GINT_SHAPE_ANY, GINT_SHAPE_2S2P1D}) {
        gint_resident_blocks(kernel_for<KVlocal>(prec, shape), 512);
        gint_resident_blocks(kernel_for<KVlocal8>(prec, shape), 512);
        gint_resident_blocks(kernel_for<KRho>(prec, shape), 256);
        gint_resident_blocks(kernel_for<KForce<false>>(prec, shape), 256);
        gint_resident_blocks(kernel_for<KForce<true>>(prec, shape), 256);
    }
}
