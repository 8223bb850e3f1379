// One SCF step on the device around the grid integrals: Gamma-point fold of
// H(R) and S(R), the generalised eigenproblem on rocSOLVER, occupations, and
// the density matrix D(R) scattered back onto the block pattern (paper: "GPU
// Acceleration of Diagonalization", Eq. 6-8).  See include/gint_scf.h.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <new>
#include <vector>

#include "gint_plan_impl.h"
#include "gint_scf.h"

hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s);

namespace {

// The pattern blocks of one atom pair (I, J), all lattice vectors R: their
// indices gblk[b_begin, b_begin + b_count) in a fixed order, and where the
// pair's n_I x n_J tile sits in the dense matrices.
struct GGroup {
    long long row, col;
    int ni, nj;
    int b_begin, b_count;
};

// dense[(row + mu) + (col + nu) n] = sum over the group's blocks of h_b[mu, nu]
// (column-major n x n; one workgroup per group, the R sum in a fixed order)
__global__ __launch_bounds__(256) void k_fold(const GGroup *__restrict__ groups, int ngroups,
                                              const int *__restrict__ gblk, const GBlk *__restrict__ blk,
                                              const double *__restrict__ h, long long n, double *__restrict__ dense) {
    for (int gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
        const GGroup g = groups[gi];
        for (int e = threadIdx.x; e < g.ni * g.nj; e += blockDim.x) {
            const int mu = e / g.nj, nu = e - mu * g.nj;
            double acc = 0.0;
            for (int q = 0; q < g.b_count; ++q) acc += h[blk[gblk[g.b_begin + q]].off + (long long)mu * g.nj + nu];
            dense[(g.row + mu) + (g.col + nu) * n] = acc;
        }
    }
}

// every block b of the pattern: d[off_b + mu n_J + nu] = dense[(row_I + mu) + (col_J + nu) n]
__global__ __launch_bounds__(256) void k_scatter(const GBlk *__restrict__ blk, int nblk,
                                                 const long long *__restrict__ orb_off, const double *__restrict__ dense,
                                                 long long n, double *__restrict__ d) {
    for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
        const GBlk k = blk[b];
        const long long r0 = orb_off[k.i], c0 = orb_off[k.j];
        for (int e = threadIdx.x; e < k.ni * k.nj; e += blockDim.x) {
            const int mu = e / k.nj, nu = e - mu * k.nj;
            d[k.off + e] = dense[(r0 + mu) + (c0 + nu) * n];
        }
    }
}

__device__ inline double fermi2(double e, double mu, double kT) { return 2.0 / (1.0 + exp((e - mu) / kT)); }

// Occupations of the n eigenvalues (ascending).  kT <= 0: aufbau, 2 per
// orbital in order until n_electrons are placed.  kT > 0: Fermi-Dirac with
// the chemical potential found by bisection (200 halvings of a bracket that
// holds every eigenvalue with 40 kT to spare).  One workgroup.
__global__ __launch_bounds__(256) void k_occupations(const double *__restrict__ e, int n, double nel, double kT,
                                                     double *__restrict__ f) {
    __shared__ double red[256];
    __shared__ double s_lo, s_hi;
    if (!(kT > 0.0)) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) f[i] = fmin(2.0, fmax(0.0, nel - 2.0 * i));
        return;
    }
    if (threadIdx.x == 0) {
        s_lo = e[0] - 40.0 * kT - 1.0;
        s_hi = e[n - 1] + 40.0 * kT + 1.0;
    }
    __syncthreads();
    for (int it = 0; it < 200; ++it) {
        const double mu = 0.5 * (s_lo + s_hi);
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) acc += fermi2(e[i], mu, kT);
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (red[0] < nel)
                s_lo = mu;
            else
                s_hi = mu;
        }
        __syncthreads();
    }
    const double mu = 0.5 * (s_lo + s_hi);
    for (int i = threadIdx.x; i < n; i += blockDim.x) f[i] = fermi2(e[i], mu, kT);
}

// zf[:, i] = z[:, i] f_i (column-major n x n)
__global__ __launch_bounds__(256) void k_scale_cols(const double *__restrict__ z, const double *__restrict__ f,
                                                    long long n, double *__restrict__ zf) {
    const long long total = n * n;
    for (long long t = blockIdx.x * 256LL + threadIdx.x; t < total; t += (long long)gridDim.x * 256)
        zf[t] = z[t] * f[t / n];
}

int grid_for(long long work) {
    const long long g = (work + 255) / 256;
    return (int)std::max(1LL, std::min(g, 8192LL));
}

}  // namespace

struct gint_scf {
    gint_plan *plan = nullptr;
    int device = 0;
    long long n = 0;
    rocblas_handle handle = nullptr;
    double *A = nullptr, *B = nullptr, *ZF = nullptr, *DG = nullptr;  // n x n each
    double *offd = nullptr;      // [n] rocSOLVER's tridiagonal work
    double *occ = nullptr;       // [n] occupations when the caller passes none
    int *info = nullptr;         // rocSOLVER status when the caller passes none
    GGroup *groups = nullptr;
    int ngroups = 0;
    int *gblk = nullptr;
    long long *orb_off = nullptr;
    GBlk *blk = nullptr;         // the plan's block table (own copy)
    int nblk = 0;
};

namespace {

void scf_release(gint_scf *s) {
    void *ptrs[] = {s->A, s->B, s->ZF, s->DG, s->offd, s->occ, s->info, s->groups, s->gblk, s->orb_off, s->blk};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s->handle) (void)rocblas_destroy_handle(s->handle);
}

int hipfail(hipError_t e) {
    gint_record_hip_error((int)e);
    return GINT_EHIP;
}

template <class T>
hipError_t put(T **dst, const std::vector<T> &v) {
    hipError_t e = hipMalloc((void **)dst, std::max<size_t>(1, v.size()) * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        return e;
    }
    if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

int check_scf_device(const gint_scf *s) {
    int cur = 0;
    const hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hipfail(e);
    return cur == s->device ? GINT_OK : GINT_EINVAL;
}

}  // namespace

extern "C" {

int gint_scf_create(gint_scf **out, gint_plan *p, int64_t *n_orbitals) {
    if (!out || !p) return GINT_EINVAL;
    if (p->n_sys != 1) return GINT_EUNSUPPORTED;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hipfail(e);
    if (cur != p->device) return GINT_EINVAL;
    gint_scf *s = new (std::nothrow) gint_scf();
    if (!s) return GINT_ENOMEM;
    s->plan = p;
    s->device = cur;
    // orbital offsets of the atoms in the dense matrices
    std::vector<long long> off(p->atom_norb.size() + 1, 0);
    for (size_t a = 0; a < p->atom_norb.size(); ++a) off[a + 1] = off[a] + p->atom_norb[a];
    s->n = off.back();
    const long long n = s->n;
    // (I, J) groups of the pattern, blocks of a group in pattern order
    std::vector<int> order(p->blocks_host.size());
    for (size_t b = 0; b < order.size(); ++b) order[b] = (int)b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const GBlk &a = p->blocks_host[x], &c = p->blocks_host[y];
        return a.i != c.i ? a.i < c.i : a.j < c.j;
    });
    std::vector<GGroup> groups;
    for (size_t k = 0; k < order.size();) {
        size_t m = k;
        const GBlk &b0 = p->blocks_host[order[k]];
        while (m < order.size() && p->blocks_host[order[m]].i == b0.i && p->blocks_host[order[m]].j == b0.j) ++m;
        groups.push_back(GGroup{off[b0.i], off[b0.j], b0.ni, b0.nj, (int)k, (int)(m - k)});
        k = m;
    }
    s->ngroups = (int)groups.size();
    s->nblk = (int)p->blocks_host.size();
    const size_t nn = (size_t)n * (size_t)n;
    int rc = GINT_OK;
    if ((e = put(&s->groups, groups)) != hipSuccess || (e = put(&s->gblk, order)) != hipSuccess ||
        (e = put(&s->orb_off, off)) != hipSuccess || (e = put(&s->blk, p->blocks_host)) != hipSuccess)
        rc = hipfail(e);
    double **mats[] = {&s->A, &s->B, &s->ZF, &s->DG};
    for (double **m : mats)
        if (rc == GINT_OK && hipMalloc((void **)m, std::max<size_t>(1, nn) * sizeof(double)) != hipSuccess) {
            *m = nullptr;
            rc = GINT_ENOMEM;
        }
    if (rc == GINT_OK && (hipMalloc((void **)&s->offd, std::max<long long>(1, n) * sizeof(double)) != hipSuccess ||
                          hipMalloc((void **)&s->occ, std::max<long long>(1, n) * sizeof(double)) != hipSuccess ||
                          hipMalloc((void **)&s->info, sizeof(int)) != hipSuccess))
        rc = GINT_ENOMEM;
    if (rc == GINT_OK && rocblas_create_handle(&s->handle) != rocblas_status_success) {
        s->handle = nullptr;
        rc = GINT_EHIP;
    }
    if (rc != GINT_OK) {
        scf_release(s);
        delete s;
        return rc;
    }
    if (n_orbitals) *n_orbitals = n;
    *out = s;
    return GINT_OK;
}

int gint_scf_fold_gamma(gint_scf *s, const double *h_vals, double *dense, void *stream) {
    if (!s || !h_vals || !dense) return GINT_EINVAL;
    if (const int rc = check_scf_device(s)) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(dense, s->n * s->n, 0.0, st);
    if (e != hipSuccess) return hipfail(e);
    if (s->ngroups > 0) {
        hipLaunchKernelGGL(k_fold, dim3(std::min(s->ngroups, 8192)), dim3(256), 0, st, s->groups, s->ngroups, s->gblk,
                           s->blk, h_vals, s->n, dense);
        if ((e = hipGetLastError()) != hipSuccess) return hipfail(e);
    }
    return GINT_OK;
}

int gint_scf_solve(gint_scf *s, const double *h_vals, const double *s_vals, double n_electrons, double kT,
                   double *eigvals, double *occupations, double *d_vals, int *info, void *stream) {
    if (!s || !h_vals || !s_vals || !eigvals || !d_vals) return GINT_EINVAL;
    if (!(n_electrons >= 0.0) || !(n_electrons <= 2.0 * (double)s->n) || !(kT == kT)) return GINT_EINVAL;
    if (s->n > 0x7fffffffLL) return GINT_EUNSUPPORTED;
    if (const int rc = check_scf_device(s)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const long long n = s->n;
    if (n == 0) return GINT_OK;
    double *f = occupations ? occupations : s->occ;
    int *inf = info ? info : s->info;
    int rc = gint_scf_fold_gamma(s, h_vals, s->A, stream);
    if (rc == GINT_OK) rc = gint_scf_fold_gamma(s, s_vals, s->B, stream);
    if (rc != GINT_OK) return rc;
    if (rocblas_set_stream(s->handle, st) != rocblas_status_success) return GINT_EHIP;
    // A <- eigenvectors Z (Z^T S Z = 1), eigvals ascending
    if (rocsolver_dsygvd(s->handle, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)n, s->A,
                         (rocblas_int)n, s->B, (rocblas_int)n, eigvals, s->offd, inf) != rocblas_status_success)
        return GINT_EHIP;
    hipLaunchKernelGGL(k_occupations, dim3(1), dim3(256), 0, st, eigvals, (int)n, n_electrons, kT, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e);
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(n * n)), dim3(256), 0, st, s->A, f, n, s->ZF);
    if ((e = hipGetLastError()) != hipSuccess) return hipfail(e);
    // D^G = (Z f) Z^T
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(s->handle, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)n, (rocblas_int)n,
                      (rocblas_int)n, &one, s->ZF, (rocblas_int)n, s->A, (rocblas_int)n, &zero, s->DG,
                      (rocblas_int)n) != rocblas_status_success)
        return GINT_EHIP;
    if (s->nblk > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(std::min(s->nblk, 8192)), dim3(256), 0, st, s->blk, s->nblk, s->orb_off,
                           s->DG, n, d_vals);
        if ((e = hipGetLastError()) != hipSuccess) return hipfail(e);
    }
    return GINT_OK;
}

void gint_scf_destroy(gint_scf *s) {
    if (!s) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    scf_release(s);
    (void)hipSetDevice(cur);
    delete s;
}

}  // extern "C"
