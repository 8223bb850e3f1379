// Device-side helpers shared by the FP64 and mixed-precision kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gint_internal.h"

// Plan descriptors (items, pairs, systems, atoms, species, bigcells) are
// never written during a launch.  Reading them through the constant address
// space tells the compiler so: a load with a wave-uniform address becomes a
// scalar load into SGPRs even after the kernel has issued global stores or
// atomics (which otherwise force vector loads inside a persistent loop).
template <class T>
using cptr = const __attribute__((address_space(4))) T *;
typedef const __attribute__((address_space(4))) GPair CPair;
typedef const __attribute__((address_space(4))) GPair8 CPair8;
typedef const __attribute__((address_space(4))) GSpecies CSpecies;
typedef const __attribute__((address_space(4))) GSys CSys;
typedef const __attribute__((address_space(4))) double cdouble;

template <class T>
__device__ inline cptr<T> cst(const T *p) {
    return (cptr<T>)p;
}

// Copy of a descriptor read through the constant address space.
template <class T>
__device__ inline T ldc(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    T v;
    int *d = reinterpret_cast<int *>(&v);
    const cptr<int> s = (cptr<int>)p;
#pragma unroll
    for (unsigned k = 0; k < sizeof(T) / 4; ++k) d[k] = s[k];
    return v;
}

// Wave index as a wave-uniform value: lets the compiler keep everything
// indexed by it (atom slots, species descriptors, channel loops) in scalar
// registers and scalar branches.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Persistent work loop: items are claimed from a device counter (reset to 0
// before every launch).  The claimed index is the same in every lane; saying
// so keeps the item's descriptor loads scalar.
__device__ inline int claim_item(int *counter, int *slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

// Geometry of system s of a batched plan into P.
__device__ inline void bind_system(GDev &P, int s) {
    CSys &S = cst(P.sys)[s];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.N[k] = S.N[k];
#pragma unroll
        for (int m = 0; m < 3; ++m) P.e[k][m] = S.e[k][m];
    }
    P.w = S.w;
}

// Channel layout of a species: with SHAPE a fixed layout (GINT_SHAPE_*) the
// channel count and each channel's l are compile-time constants, so the
// orbital evaluation unrolls completely (orbital slots and LDS offsets become
// constants and no per-channel branches remain); SHAPE 0 reads them from the
// species record.
template <int SHAPE>
struct ChanShape {
    __device__ static int nchan(CSpecies &sp) { return sp.nchan; }
    __device__ static int l(CSpecies &sp, int c) { return sp.chan_l[c]; }
};
template <>
struct ChanShape<GINT_SHAPE_2S2P1D> {
    __device__ static constexpr int nchan(CSpecies &) { return 5; }
    __device__ static constexpr int l(CSpecies &, int c) { return c < 2 ? 0 : (c < 4 ? 1 : 2); }
    static constexpr int norb = 13;
};
template <>
struct ChanShape<GINT_SHAPE_2S1P> {
    __device__ static constexpr int nchan(CSpecies &) { return 3; }
    __device__ static constexpr int l(CSpecies &, int c) { return c < 2 ? 0 : 1; }
    static constexpr int norb = 5;
};

// f(std::integral_constant<int, SHAPE>) for the species' layout (a
// wave-uniform branch on the species record).
template <class F>
__device__ __attribute__((always_inline)) inline void by_shape(CSpecies &sp, F &&f) {
    const int shape = sp.shape;
    if (shape == GINT_SHAPE_2S2P1D)
        f(std::integral_constant<int, GINT_SHAPE_2S2P1D>{});
    else if (shape == GINT_SHAPE_2S1P)
        f(std::integral_constant<int, GINT_SHAPE_2S1P>{});
    else
        f(std::integral_constant<int, GINT_SHAPE_ANY>{});
}

// As by_shape, for a kernel compiled for plans whose species all have layout
// KS (then no branch remains), or for any mix (KS = GINT_SHAPE_ANY).
template <int KS, class F>
__device__ __attribute__((always_inline)) inline void with_shape(CSpecies &sp, F &&f) {
    if constexpr (KS != GINT_SHAPE_ANY)
        f(std::integral_constant<int, KS>{});
    else
        by_shape(sp, f);
}

