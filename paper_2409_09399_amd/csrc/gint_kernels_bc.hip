// Bigcell-stationary rho and force/stress, mixed precision (gfx950).
//
// The cluster-pair kernels evaluate an atom's orbitals once for every
// cluster pair whose region covers a bigcell, which on the bilayer workloads
// means each (point, orbital) value is computed tens of times.  Here one
// workgroup owns a brick of bigcells (gint_internal.h): for each bigcell it
// finds the atom images active on its 64 points, evaluates their orbitals
// once into LDS, and forms
//
//     psi_J[p, nu] = sum_{I, mu} phi_I[p, mu] D_sym(I, J, T_J - T_I)[mu, nu]   (Eq. 3, 4)
//
// for every active image J on FP16/BF16 MFMA (hi/lo split operands, three
// products, FP32 accumulation over all I).  Then per point p (one lane):
//     rho_p  = sum_J phi_J(p) . psi_J(p)                      (written once, no atomics)
//     F_J   += 2 w V_p grad phi_J(p) . psi_J(p),  Z += 2 w V_p grad phi_J x^T . psi_J,
//     E     += w V_p rho_p                                     (Eq. 4-5)
// with the per-point terms in FP32 and every sum across points in FP64.
// D_sym enters as a per-call 16-bit hi/lo copy in MFMA operand order
// (k_d16), scaled by one power of two so that its largest entry maps below
// 2^13 (the split then stays clear of the FP16 subnormal range).
#include <hip/hip_runtime.h>

#include "gint_mixed.h"

namespace {

constexpr int BC_WAVES = 8;                 // waves of a rho/force workgroup
constexpr int BC_THREADS = 64 * BC_WAVES;
constexpr int BC_CI = 8;                    // I images per staged chunk (four 32-wide k-steps), one per wave
constexpr int BC_ROW = 16 * BC_CI + 8;      // 16-bit elements per point row of the chunk tile
// J images per wave in one J group (their psi accumulators stay in
// registers through the group): three for rho, two for the force pass,
// whose per-point gradient code needs more registers.  With these the
// kernels fit about 128 VGPRs, so that two workgroups (four waves per SIMD)
// share a CU and hide each other's table and D latency; measured on the
// bilayer, more J per wave spills and fewer re-evaluates phi more often.
template <bool FORCE>
constexpr int bc_jw() {
    return FORCE ? 2 : 3;
}
constexpr int BC_PSTR = 17;                 // floats per point row of a wave's psi buffer

// D_sym of pattern block b as 16-bit hi/lo, scaled by sD, in the order the
// B operand of v_mfma_f32_16x16x32 reads it: [nu][mu] (column nu of the
// block is contiguous), 16 x 16 with zero padding; hi then lo, 1 KiB a block.
template <class T>
__global__ __launch_bounds__(256) void k_d16(const GBlk *__restrict__ blk, int nblk, const double *__restrict__ D,
                                             const double *__restrict__ dmax, unsigned short *__restrict__ d16) {
    const float sD = pow2_scale(*dmax);
    const int e = threadIdx.x, nu = e >> 4, mu = e & 15;
    for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
        const GBlk k = ldc(blk + b);
        float v = 0.f;
        if (mu < k.ni && nu < k.nj) {
            const double s = 0.5 * (D[k.off + (long long)mu * k.nj + nu] + D[k.off_t + (long long)nu * k.ni + mu]);
            v = (float)(s * (double)sD);
        }
        T hi, lo;
        Split16<T>::split(v, hi, lo);
        unsigned short *o = d16 + (size_t)b * 512;
        o[nu * 16 + mu] = __builtin_bit_cast(unsigned short, hi);
        o[256 + nu * 16 + mu] = __builtin_bit_cast(unsigned short, lo);
    }
}

// Position and species of union image i as a Slot (disp_at's input).
__device__ inline Slot uslot(const GUAtom *U, int i) {
    const GUAtom u = ldc(U + i);
    return Slot{u.x, u.y, u.z, u.species};
}

// A value every lane holds the same copy of, as a wave-uniform (scalar) one.
__device__ inline unsigned long long uniform64(unsigned long long v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// One (point, image) row of the chunk tile: 16 hi and 16 lo values of the
// image's orbitals (scaled by sphi), zeros where the image is inactive.
template <class T, int KS>
__device__ __attribute__((always_inline)) inline void stage_row(const GDev &P, const P3 &r, const Slot &s, float sphi,
                                                                 T *h0, T *h1) {
    const Disp d = disp_at(P, r, s);
    if (d.in) {
        CSpecies &sp = cst(P.species)[s.species];
        with_shape<KS>(sp, [&](auto shp) {
            constexpr int SH = decltype(shp)::value;
            if constexpr (SH != GINT_SHAPE_ANY) {
                stage_b16_rows<T, SH>(sp, P.tab32, d, sphi, h0, h1);
            } else {
                eval32<SH>(sp, P.tab32, d.x, d.y, d.z, d.kn, sphi, [&](int mu, float v) {
                    T hi, lo;
                    Split16<T>::split(v, hi, lo);
                    h0[mu] = hi;
                    h1[mu] = lo;
                });
            }
        });
    } else {
        const u4v z = {0u, 0u, 0u, 0u};
        *(u4v *)h0 = z;
        *(u4v *)(h0 + 8) = z;
        *(u4v *)h1 = z;
        *(u4v *)(h1 + 8) = z;
    }
}

// Work claim with one queue per XCD.  The bricks are in spatial order; queue
// q holds the q-th eighth of the list, and workgroup b (which the dispatcher
// places on XCD b mod 8) serves queue b mod 8 first, so the bricks an XCD
// works on at any time are neighbours and share their D blocks in that XCD's
// L2.  An exhausted queue is remembered in *done; then the other queues are
// served in turn.  Returns -1 when every queue is empty.  counters: eight
// ints, zero at launch.
__device__ inline int claim_brick(int *counters, int nbricks, int *slot, unsigned *done) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const int x = blockIdx.x & 7;
        int got = -1;
        for (int k = 0; k < 8 && got < 0; ++k) {
            const int q = (x + k) & 7;
            if ((*done >> q) & 1u) continue;
            const int b0 = (int)((long long)nbricks * q / 8), b1 = (int)((long long)nbricks * (q + 1) / 8);
            const int i = b1 > b0 ? atomicAdd(counters + q, 1) : 0;
            if (i < b1 - b0)
                got = b0 + i;
            else
                *done |= 1u << q;
        }
        *slot = got;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

}  // namespace

// ---------------------------------------------------------------------------
// rho (FORCE = false) or force/stress/E (FORCE = true, with rho when RHO),
// one brick per claimed work item.
// ---------------------------------------------------------------------------
template <class T, int KS, bool FORCE, bool RHO>
__global__ __launch_bounds__(BC_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_bc_mx(GDev P0, const double *__restrict__ V0, double *__restrict__ F,
                                                  double *__restrict__ ZE0, double *__restrict__ rho0) {
    typedef Split16<T> S;
    typedef typename S::vec vec;
    constexpr bool WRHO = !FORCE || RHO;
    constexpr int BC_JW = bc_jw<FORCE>();   // J images per wave in one J group
    constexpr int BC_JG = BC_WAVES * BC_JW;  // J images per J group (round-robin over the waves)
    __shared__ __attribute__((aligned(16))) T tA[2][GINT_BCPTS][BC_ROW];
    // a wave's psi rows; after the last J group, its 64 rho partials (FP64)
    __shared__ __attribute__((aligned(16))) float psb[BC_WAVES][GINT_BCPTS * BC_PSTR];
    __shared__ unsigned long long act[GINT_UMAX];
    __shared__ short lst[GINT_UMAX];
    __shared__ double fbuf[FORCE ? GINT_UMAX : 1][3];
    __shared__ double zred[BC_WAVES][10];
    __shared__ int s_nact;
    __shared__ int s_item;
    __shared__ unsigned s_done;
    const int lane = threadIdx.x & 63, w = wave_id();
    const float sphi = (float)P0.phi_scale;
    const float unscale = 1.f / (sphi * pow2_scale(*cst(P0.dmax)));
    const unsigned short *__restrict__ d16 = P0.d16;
    if (threadIdx.x == 0) s_done = 0u;
    for (;;) {
        const int item_ = claim_brick(P0.counter, P0.nbricks, &s_item, &s_done);
        if (item_ < 0) break;
        const GBrick bk = ldc(P0.bricks + item_);
        GDev P = P0;
        bind_system(P, bk.sys);
        CSys &SY = cst(P0.sys)[bk.sys];
        const int n = bk.u_count;
        const GUAtom *U = P0.uatoms + bk.u_begin;
        const cptr<int> pt = cst(P0.ptab + bk.pt_off);
        double z9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, en = 0.0;
        if constexpr (FORCE) {
            for (int i = threadIdx.x; i < n; i += BC_THREADS) fbuf[i][0] = fbuf[i][1] = fbuf[i][2] = 0.0;
        }
        for (int s0 = 0; s0 < bk.nb[0]; ++s0)
        for (int s1 = 0; s1 < bk.nb[1]; ++s1)
        for (int s2 = 0; s2 < bk.nb[2]; ++s2) {
            // this lane's point of the bigcell
            const int n0 = bk.o[0] + 4 * s0 + (lane >> 4), n1 = bk.o[1] + 4 * s1 + ((lane >> 2) & 3),
                      n2 = bk.o[2] + 4 * s2 + (lane & 3);
            const bool inside = n0 < P.N[0] && n1 < P.N[1] && n2 < P.N[2];
            P3 r;
            r.x = n0 * P.e[0][0] + n1 * P.e[1][0] + n2 * P.e[2][0];
            r.y = n0 * P.e[0][1] + n1 * P.e[1][1] + n2 * P.e[2][1];
            r.z = n0 * P.e[0][2] + n1 * P.e[1][2] + n2 * P.e[2][2];
            r.g = inside ? ((long long)n0 * P.N[1] + n1) * P.N[2] + n2 : 0;
            double vpt = 0.0;
            if (FORCE && inside) vpt = V0[SY.g_off + r.g];
            // phase 1: activity of every union image on the 64 points
            for (int i = w; i < n; i += BC_WAVES) {
                const unsigned long long m = __ballot(inside && reaches(P, r, uslot(U, i)));
                if (lane == 0) act[i] = m;
            }
            __syncthreads();
            // compact list of the active images (wave 0, in union order)
            if (w == 0) {
                int cnt = 0;
                for (int base = 0; base < n; base += 64) {
                    const int i = base + lane;
                    const bool f = i < n && act[i] != 0ull;
                    const unsigned long long b = __ballot(f);
                    const int pos = cnt + __builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0));
                    if (f) lst[pos] = (short)i;
                    cnt += __popcll(b);
                }
                if (lane == 0) s_nact = cnt;
            }
            __syncthreads();
            const int nact = __builtin_amdgcn_readfirstlane(s_nact);
            double racc = 0.0;
            for (int jg = 0; jg < nact; jg += BC_JG) {
                f4v c[BC_JW][4];
#pragma unroll
                for (int jj = 0; jj < BC_JW; ++jj)
#pragma unroll
                    for (int t = 0; t < 4; ++t) c[jj][t] = (f4v){0.f, 0.f, 0.f, 0.f};
                for (int ic = 0; ic < nact; ic += BC_CI) {
                    // pair-table entries of the chunk's I images and the wave's J
                    // images, one per lane (lane 8 q + jj: I image ic + q, J image
                    // jg + w + BC_WAVES jj), loaded before the stage so that their
                    // latency is hidden behind it
                    int ptv = -1;
                    {
                        const int ix = ic + (lane >> 3), jx = jg + w + BC_WAVES * (lane & 7);
                        if ((lane & 7) < BC_JW && ix < nact && jx < nact)
                            ptv = P0.ptab[bk.pt_off + (long long)lst[ix] * n + lst[jx]];
                    }
                    // stage the chunk: wave w writes slot w
                    {
                        const int slot = w, idx = ic + slot;
                        T *h0 = &tA[0][lane][slot * 16];
                        T *h1 = &tA[1][lane][slot * 16];
                        if (idx < nact) {
                            const int i = __builtin_amdgcn_readfirstlane((int)lst[idx]);
                            stage_row<T, KS>(P, r, uslot(U, i), sphi, h0, h1);
                        } else {
                            const u4v z = {0u, 0u, 0u, 0u};
                            *(u4v *)h0 = z;
                            *(u4v *)(h0 + 8) = z;
                            *(u4v *)h1 = z;
                            *(u4v *)(h1 + 8) = z;
                        }
                    }
                    __syncthreads();
                    // psi_J += phi_chunk D_sym(chunk, J) for the wave's J images, one
                    // 32-wide k-step (two I images) at a time: the step's B operands
                    // of every J are requested first, then each A fragment is read
                    // from LDS once and serves all the wave's J
                    int jv[BC_JW];
                    unsigned long long mjv[BC_JW];
#pragma unroll
                    for (int jj = 0; jj < BC_JW; ++jj) {
                        const int jidx = jg + w + BC_WAVES * jj;
                        jv[jj] = jidx < nact ? __builtin_amdgcn_readfirstlane((int)lst[jidx]) : -1;
                        mjv[jj] = jv[jj] >= 0 ? uniform64(act[jv[jj]]) : 0ull;
                    }
#pragma unroll
                    for (int s = 0; s < BC_CI / 2; ++s) {
                        const int i0x = ic + 2 * s, i1x = i0x + 1;
                        if (i0x >= nact) break;
                        const int i0 = __builtin_amdgcn_readfirstlane((int)lst[i0x]);
                        const int i1 = i1x < nact ? __builtin_amdgcn_readfirstlane((int)lst[i1x]) : -1;
                        const unsigned long long mi = uniform64(act[i0] | (i1 >= 0 ? act[i1] : 0ull));
                        vec bh[BC_JW], blo[BC_JW];
                        unsigned long long mm[BC_JW];
                        unsigned long long any = 0ull;
#pragma unroll
                        for (int jj = 0; jj < BC_JW; ++jj) {
                            const int b0 = __builtin_amdgcn_readlane(ptv, 16 * s + jj);
                            const int b1 = i1 >= 0 ? __builtin_amdgcn_readlane(ptv, 16 * s + 8 + jj) : -1;
                            mm[jj] = (b0 >= 0 || b1 >= 0) ? (mi & mjv[jj]) : 0ull;
                            any |= mm[jj];
                            const int bl = lane < 32 ? b0 : b1;
                            if (mm[jj] != 0ull && bl >= 0) {
                                const unsigned short *src =
                                    d16 + (size_t)bl * 512 + (lane & 15) * 16 + 8 * ((lane >> 4) & 1);
                                bh[jj] = *(const vec *)src;
                                blo[jj] = *(const vec *)(src + 256);
                            } else {
#pragma unroll
                                for (int e = 0; e < 8; ++e) {
                                    bh[jj][e] = (T)0.f;
                                    blo[jj][e] = (T)0.f;
                                }
                            }
                        }
                        if (any == 0ull) continue;
                        const int col = (2 * s + (lane >> 5)) * 16 + 8 * ((lane >> 4) & 1);
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            if (!((any >> (16 * t)) & 0xFFFFull)) continue;
                            const vec ah = *(const vec *)&tA[0][16 * t + (lane & 15)][col];
                            const vec al = *(const vec *)&tA[1][16 * t + (lane & 15)][col];
#pragma unroll
                            for (int jj = 0; jj < BC_JW; ++jj) {
                                if (!((mm[jj] >> (16 * t)) & 0xFFFFull)) continue;
                                c[jj][t] = S::mfma(ah, bh[jj], c[jj][t]);
                                c[jj][t] = S::mfma(ah, blo[jj], c[jj][t]);
                                c[jj][t] = S::mfma(al, bh[jj], c[jj][t]);
                            }
                        }
                    }
                    __syncthreads();
                }
                // per point: the wave's J images against their psi
                float *ps = psb[w];
#pragma unroll
                for (int jj = 0; jj < BC_JW; ++jj) {
                    const int jidx = jg + w + BC_WAVES * jj;
                    if (jidx >= nact) break;
                    const int j = __builtin_amdgcn_readfirstlane((int)lst[jidx]);
                    const unsigned long long mj = uniform64(act[j]);
                    // psi_J to point rows (MFMA layout: lane l, register q holds
                    // point 16 t + 4 (l >> 4) + q, orbital l & 15)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (!((mj >> (16 * t)) & 0xFFFFull)) continue;
                        float *dst = ps + (16 * t + 4 * (lane >> 4)) * BC_PSTR + (lane & 15);
#pragma unroll
                        for (int q = 0; q < 4; ++q) dst[q * BC_PSTR] = c[jj][t][q] * unscale;
                    }
                    const Slot sj = uslot(U, j);
                    const Disp d = disp_at(P, r, sj);
                    const bool on = inside && d.in;
                    double f3[3] = {0.0, 0.0, 0.0};
                    if (on) {
                        CSpecies &sp = cst(P.species)[sj.species];
                        const float *prow = ps + lane * BC_PSTR;
                        if constexpr (!FORCE) {
                            float v = 0.f;
                            with_shape<KS>(sp, [&](auto shp) {
                                constexpr int SH = decltype(shp)::value;
                                eval32<SH>(sp, P.tab32, d.x, d.y, d.z, d.kn, 1.f, [&](int mu, float x) {
                                    if constexpr (SH != GINT_SHAPE_ANY)
                                        if (mu >= ChanShape<SH>::norb) return;
                                    v += x * prow[mu];
                                });
                            });
                            racc += (double)v;
                        } else {
                            const float rr = ((float)d.kn.k + d.kn.t) * (float)sp.dr;
                            float e, G[3];
                            with_shape<KS>(sp, [&](auto shp) {
                                dot_grad32<decltype(shp)::value>(sp, P.tab32, d.x, d.y, d.z, d.kn,
                                                                 rr > 0.f ? __builtin_amdgcn_rcpf(rr) : 0.f, prow, e, G);
                            });
                            const double wv = P.w * vpt, c2 = 2.0 * wv;
                            const double gs[3] = {G[0], G[1], G[2]}, xs[3] = {d.x, d.y, d.z};
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                f3[a] = c2 * gs[a];
#pragma unroll
                                for (int b = 0; b < 3; ++b) z9[3 * a + b] += c2 * gs[a] * xs[b];
                            }
                            en += wv * (double)e;
                            if (RHO) racc += (double)e;
                        }
                    }
                    if constexpr (FORCE) {
                        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
                            for (int a = 0; a < 3; ++a) f3[a] += __shfl_xor(f3[a], off);
                        }
                        if (lane == 0) {
                            fbuf[j][0] += f3[0];
                            fbuf[j][1] += f3[1];
                            fbuf[j][2] += f3[2];
                        }
                    }
                }
            }
            if constexpr (WRHO) {
                // the partials go into the wave's own psi buffer, which only
                // this wave has used since the last barrier
                ((double *)psb[w])[lane] = racc;
                __syncthreads();
                if (w == 0 && inside) {
                    double q[BC_WAVES];
#pragma unroll
                    for (int k = 0; k < BC_WAVES; ++k) q[k] = ((const double *)psb[k])[lane];
#pragma unroll
                    for (int h = 1; h < BC_WAVES; h *= 2)
#pragma unroll
                        for (int k = 0; k < BC_WAVES; k += 2 * h) q[k] += q[k + h];
                    rho0[SY.g_off + r.g] = q[0];
                }
            }
            __syncthreads();
        }
        if constexpr (FORCE) {
            // forces of the brick's images, then Z and E of the workgroup's points
            for (int i = threadIdx.x; i < n; i += BC_THREADS) {
                const int a = U[i].atom;
                if (fbuf[i][0] != 0.0 || fbuf[i][1] != 0.0 || fbuf[i][2] != 0.0) {
                    atomicAdd(F + 3 * a + 0, fbuf[i][0]);
                    atomicAdd(F + 3 * a + 1, fbuf[i][1]);
                    atomicAdd(F + 3 * a + 2, fbuf[i][2]);
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
                for (int a = 0; a < 9; ++a) z9[a] += __shfl_xor(z9[a], off);
                en += __shfl_xor(en, off);
            }
            if (lane == 0) {
#pragma unroll
                for (int a = 0; a < 9; ++a) zred[w][a] = z9[a];
                zred[w][9] = en;
            }
            __syncthreads();
            if (threadIdx.x < 10) {
                const int k = threadIdx.x;
                double q[BC_WAVES];
#pragma unroll
                for (int u = 0; u < BC_WAVES; ++u) q[u] = zred[u][k];
#pragma unroll
                for (int h = 1; h < BC_WAVES; h *= 2)
#pragma unroll
                    for (int u = 0; u < BC_WAVES; u += 2 * h) q[u] += q[u + h];
                const double v = q[0];
                if (v != 0.0) atomicAdd(ZE0 + 10 * bk.sys + k, v);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// H_IJR (Eq. 2), mixed precision, bigcell-stationary.  The brick's union is
// cut into chunks of eight images; for each chunk pair (a <= b) the
// workgroup sweeps the brick's bigcells, staging phi of chunk a (the MFMA A
// operand, [slot][orbital][point]) and V phi of chunk b (B operand), and
// accumulates the 8 x 8 tiles H(i, j) = sum_p phi_i(p) V_p phi_j(p) in FP32
// registers across the brick (each wave owns the tiles of two i images).
// Then every tile is added once to its pattern block (I_i, J_j, T_j - T_i)
// and, for i != j, transposed to (J_j, I_i, T_i - T_j), with FP64 atomics.
// Tiles of a chunk with itself are computed for i <= j only.
// ---------------------------------------------------------------------------
constexpr int BV_C = 8;   // images per chunk

template <class T, int KS>
__global__ __launch_bounds__(256, 2) void k_bcv_mx(GDev P0, const GBlk *__restrict__ blk, const double *__restrict__ V0,
                                                   double *__restrict__ H) {
    typedef Split16<T> S;
    typedef typename S::vec vec;
    __shared__ __attribute__((aligned(16))) T tA[2][BV_C][16][TSTR];
    __shared__ __attribute__((aligned(16))) T tB[2][BV_C][16][TSTR];
    __shared__ unsigned long long actA[BV_C], actB[BV_C];
    __shared__ int s_item;
    __shared__ unsigned s_done;
    const int lane = threadIdx.x & 63, w = wave_id();
    // A = phi sphi, B = V phi sB, both below 2^13 in magnitude
    const float sphi = (float)P0.phi_scale;
    const float sB = pow2_scale(*cst(P0.vmax) * (8192.0 / P0.phi_scale));
    const double unscale = 1.0 / ((double)sphi * (double)sB);
    if (threadIdx.x == 0) s_done = 0u;
    for (;;) {
        const int item_ = claim_brick(P0.counter, P0.nbricks, &s_item, &s_done);
        if (item_ < 0) break;
        const GBrick bk = ldc(P0.bricks + item_);
        GDev P = P0;
        bind_system(P, bk.sys);
        CSys &SY = cst(P0.sys)[bk.sys];
        const int n = bk.u_count;
        const GUAtom *U = P0.uatoms + bk.u_begin;
        const cptr<int> pt = cst(P0.ptab + bk.pt_off);
        const double *V = V0 + SY.g_off;
        const int nch = (n + BV_C - 1) / BV_C;
        for (int ca = 0; ca < nch; ++ca)
        for (int cb = ca; cb < nch; ++cb) {
            f4v c[2][BV_C];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int jb = 0; jb < BV_C; ++jb) c[a][jb] = (f4v){0.f, 0.f, 0.f, 0.f};
            unsigned touched = 0u;   // bit 8 a + jb: the tile got a product
            for (int s0 = 0; s0 < bk.nb[0]; ++s0)
            for (int s1 = 0; s1 < bk.nb[1]; ++s1)
            for (int s2 = 0; s2 < bk.nb[2]; ++s2) {
                const int n0 = bk.o[0] + 4 * s0 + (lane >> 4), n1 = bk.o[1] + 4 * s1 + ((lane >> 2) & 3),
                          n2 = bk.o[2] + 4 * s2 + (lane & 3);
                const bool inside = n0 < P.N[0] && n1 < P.N[1] && n2 < P.N[2];
                P3 r;
                r.x = n0 * P.e[0][0] + n1 * P.e[1][0] + n2 * P.e[2][0];
                r.y = n0 * P.e[0][1] + n1 * P.e[1][1] + n2 * P.e[2][1];
                r.z = n0 * P.e[0][2] + n1 * P.e[1][2] + n2 * P.e[2][2];
                r.g = inside ? ((long long)n0 * P.N[1] + n1) * P.N[2] + n2 : 0;
                const float vg = inside ? (float)V[r.g] * sB : 0.f;
                // stage: wave w writes slots 2w and 2w+1 of both tiles
#pragma unroll
                for (int side = 0; side < 2; ++side) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int slot = 2 * w + q;
                        const int idx = (side == 0 ? ca : cb) * BV_C + slot;
                        T(*tile)[BV_C][16][TSTR] = side == 0 ? tA : tB;
                        unsigned long long *act = side == 0 ? actA : actB;
                        if (idx >= n) {
                            if (lane == 0) act[slot] = 0ull;
                            continue;
                        }
                        const Slot su = uslot(U, idx);
                        const Disp d = disp_at(P, r, su);
                        const bool in = inside && d.in;
                        const unsigned long long m = __ballot(in);
                        if (lane == 0) act[slot] = m;
                        // taken by every lane, before the branch: a ballot inside
                        // the inactive branch would see only inactive lanes
                        const bool zero_half = half_active(in);
                        if (in) {
                            CSpecies &sp = cst(P.species)[su.species];
                            const float scale = side == 0 ? sphi : vg;
                            with_shape<KS>(sp, [&](auto shp) {
                                constexpr int SH = decltype(shp)::value;
                                eval32<SH>(sp, P.tab32, d.x, d.y, d.z, d.kn, scale, [&](int mu, float v) {
                                    T hi, lo;
                                    if constexpr (SH != GINT_SHAPE_ANY) {
                                        // padding rows reach only output rows or columns
                                        // beyond the orbital count, which are never stored
                                        if (mu >= ChanShape<SH>::norb) return;
                                        S::split_mix(v, hi, lo);
                                    } else {
                                        S::split(v, hi, lo);
                                    }
                                    tile[0][slot][mu][lane] = hi;
                                    tile[1][slot][mu][lane] = lo;
                                });
                            });
                        } else if (zero_half) {
                            // zeros only where a 32-point k-step of this slot is read
#pragma unroll
                            for (int mu = 0; mu < rows_used<KS>(); ++mu) {
                                tile[0][slot][mu][lane] = (T)0.f;
                                tile[1][slot][mu][lane] = (T)0.f;
                            }
                        }
                    }
                }
                __syncthreads();
                const int row = lane & 15, col = 8 * (lane >> 4);
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int il = 2 * w + a;
                    if (ca * BV_C + il >= n) continue;
                    const unsigned long long mi = uniform64(actA[il]);
                    if (mi == 0ull) continue;
#pragma unroll
                    for (int jb = 0; jb < BV_C; ++jb) {
                        if (cb * BV_C + jb >= n) break;
                        if (ca == cb && jb < il) continue;
                        const unsigned long long mm = mi & uniform64(actB[jb]);
#pragma unroll
                        for (int kk = 0; kk < 2; ++kk) {
                            if (!((mm >> (32 * kk)) & 0xffffffffull)) continue;
                            const vec ahi = *(const vec *)&tA[0][il][row][32 * kk + col];
                            const vec alo = *(const vec *)&tA[1][il][row][32 * kk + col];
                            const vec bhi = *(const vec *)&tB[0][jb][row][32 * kk + col];
                            const vec blo = *(const vec *)&tB[1][jb][row][32 * kk + col];
                            c[a][jb] = S::mfma(ahi, bhi, c[a][jb]);
                            c[a][jb] = S::mfma(ahi, blo, c[a][jb]);
                            c[a][jb] = S::mfma(alo, bhi, c[a][jb]);
                            touched |= 1u << (8 * a + jb);
                        }
                    }
                }
                __syncthreads();
            }
            // 16x16x32 result layout: lane l, register q holds row 4 (l >> 4) + q, column l & 15
            const int nu = lane & 15;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
                for (int jb = 0; jb < BV_C; ++jb) {
                    if (!((touched >> (8 * a + jb)) & 1u)) continue;
                    const int i = ca * BV_C + 2 * w + a, j = cb * BV_C + jb;
                    const int b = pt[(long long)i * n + j];
                    const int bt = i != j ? pt[(long long)j * n + i] : -1;
                    if (b >= 0) {
                        const GBlk k = ldc(blk + b);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int mu = 4 * (lane >> 4) + q;
                            if (mu < k.ni && nu < k.nj)
                                atomicAdd(H + k.off + (long long)mu * k.nj + nu, P.w * unscale * (double)c[a][jb][q]);
                        }
                    }
                    if (bt >= 0) {
                        const GBlk k = ldc(blk + bt);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int mu = 4 * (lane >> 4) + q;
                            if (mu < k.nj && nu < k.ni)
                                atomicAdd(H + k.off + (long long)nu * k.nj + mu, P.w * unscale * (double)c[a][jb][q]);
                        }
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int gint_persistent_grid(const void *kernel, int nitems, int threads);
int gint_resident_blocks(const void *kernel, int threads);
hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s);
hipError_t gint_launch_absmax(const double *x, long long n, double *out, hipStream_t s);

namespace {

template <class T, int KS, bool FORCE, bool RHO>
const void *bc_kernel() {
    return (const void *)k_bc_mx<T, KS, FORCE, RHO>;
}

template <bool FORCE, bool RHO>
const void *bc_kernel_for(int prec, int shape_all) {
    const bool fixed = shape_all == GINT_SHAPE_2S2P1D;
    if (prec == 2)
        return fixed ? bc_kernel<__bf16, GINT_SHAPE_2S2P1D, FORCE, RHO>() : bc_kernel<__bf16, GINT_SHAPE_ANY, FORCE, RHO>();
    return fixed ? bc_kernel<_Float16, GINT_SHAPE_2S2P1D, FORCE, RHO>() : bc_kernel<_Float16, GINT_SHAPE_ANY, FORCE, RHO>();
}

}  // namespace

// max |D| into P.dmax, then D_sym as 16-bit hi/lo into P.d16
hipError_t gint_launch_d16(const GDev &P, int prec, const GBlk *blocks, long long nnz, const double *D, hipStream_t s) {
    hipError_t e = gint_launch_fill(const_cast<double *>(P.dmax), 1, 0.0, s);
    if (e == hipSuccess) e = gint_launch_absmax(D, nnz, const_cast<double *>(P.dmax), s);
    if (e != hipSuccess || P.nblocks <= 0) return e;
    const int grid = P.nblocks < 8192 ? P.nblocks : 8192;
    unsigned short *d16 = const_cast<unsigned short *>(P.d16);
    if (prec == 2)
        hipLaunchKernelGGL(k_d16<__bf16>, dim3(grid), dim3(256), 0, s, blocks, P.nblocks, D, P.dmax, d16);
    else
        hipLaunchKernelGGL(k_d16<_Float16>, dim3(grid), dim3(256), 0, s, blocks, P.nblocks, D, P.dmax, d16);
    return hipGetLastError();
}

namespace {

hipError_t launch_bc(const void *k, const GDev &P, hipStream_t s, const double *V, double *F, double *ZE, double *rho) {
    if (P.nbricks <= 0) return hipSuccess;
    hipError_t e = gint_launch_fill((double *)P.counter, 4, 0.0, s);   // the eight queue counters
    if (e != hipSuccess) return e;
    const int grid = gint_persistent_grid(k, P.nbricks, BC_THREADS);
    void *argv[] = {const_cast<GDev *>(&P), &V, &F, &ZE, &rho};
    e = hipLaunchKernel(k, dim3(grid), dim3(BC_THREADS), argv, 0, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace

// rho (mixed forms, bigcell-stationary).  rho must be cleared by the caller
// (points of bricks no atom reaches are not written).
hipError_t gint_launch_rho_bc_prepared(const GDev &P, int prec, double *rho, hipStream_t s) {
    return launch_bc(bc_kernel_for<false, false>(prec, P.shape_all), P, s, nullptr, nullptr, nullptr, rho);
}

hipError_t gint_launch_rho_bc(const GDev &P, int prec, const GBlk *blocks, long long nnz, const double *D,
                              double *rho, hipStream_t s) {
    hipError_t e = gint_launch_d16(P, prec, blocks, nnz, D, s);
    if (e != hipSuccess) return e;
    return gint_launch_rho_bc_prepared(P, prec, rho, s);
}

// force/stress/E (and rho when given; rho cleared by the caller).  F and ZE
// cleared by the caller.
hipError_t gint_launch_force_bc_prepared(const GDev &P, int prec, const double *V, double *F, double *ZE, double *rho,
                                         hipStream_t s) {
    if (rho) return launch_bc(bc_kernel_for<true, true>(prec, P.shape_all), P, s, V, F, ZE, rho);
    return launch_bc(bc_kernel_for<true, false>(prec, P.shape_all), P, s, V, F, ZE, nullptr);
}

hipError_t gint_launch_force_bc(const GDev &P, int prec, const GBlk *blocks, long long nnz, const double *V,
                                const double *D, double *F, double *ZE, double *rho, hipStream_t s) {
    hipError_t e = gint_launch_d16(P, prec, blocks, nnz, D, s);
    if (e != hipSuccess) return e;
    return gint_launch_force_bc_prepared(P, prec, V, F, ZE, rho, s);
}

// H (mixed forms, bigcell-stationary): P.vmax must hold max |V| of this call
// and H must be cleared by the caller.
hipError_t gint_launch_vlocal_bc(const GDev &P, int prec, const GBlk *blocks, const double *V, double *H,
                                 hipStream_t s) {
    if (P.nbricks <= 0) return hipSuccess;
    const bool fixed = P.shape_all == GINT_SHAPE_2S2P1D;
    const void *k = prec == 2 ? (fixed ? (const void *)k_bcv_mx<__bf16, GINT_SHAPE_2S2P1D>
                                       : (const void *)k_bcv_mx<__bf16, GINT_SHAPE_ANY>)
                              : (fixed ? (const void *)k_bcv_mx<_Float16, GINT_SHAPE_2S2P1D>
                                       : (const void *)k_bcv_mx<_Float16, GINT_SHAPE_ANY>);
    hipError_t e = gint_launch_fill((double *)P.counter, 4, 0.0, s);   // the eight queue counters
    if (e != hipSuccess) return e;
    const int grid = gint_persistent_grid(k, P.nbricks, 256);
    void *argv[] = {const_cast<GDev *>(&P), &blocks, &V, &H};
    e = hipLaunchKernel(k, dim3(grid), dim3(256), argv, 0, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

void gint_prime_grids_bc(int prec) {
    for (int shape : {GINT_SHAPE_ANY, GINT_SHAPE_2S2P1D}) {
        gint_resident_blocks(bc_kernel_for<false, false>(prec, shape), BC_THREADS);
        gint_resident_blocks(bc_kernel_for<true, false>(prec, shape), BC_THREADS);
        gint_resident_blocks(bc_kernel_for<true, true>(prec, shape), BC_THREADS);
    }
    if (prec == 2) {
        gint_resident_blocks((const void *)k_bcv_mx<__bf16, GINT_SHAPE_2S2P1D>, 256);
        gint_resident_blocks((const void *)k_bcv_mx<__bf16, GINT_SHAPE_ANY>, 256);
    } else {
        gint_resident_blocks((const void *)k_bcv_mx<_Float16, GINT_SHAPE_2S2P1D>, 256);
        gint_resident_blocks((const void *)k_bcv_mx<_Float16, GINT_SHAPE_ANY>, 256);
    }
}
