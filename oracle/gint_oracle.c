/* FP64 CPU oracle for real-space grid integration.  TEST INFRASTRUCTURE
 * ONLY: loaded by the tests, the smoke check and the benchmark's CPU
 * baseline, never by the product path.  Shares no code with the HIP library.
 *
 * Every routine follows the plain definitions restated in gint_oracle.h
 * (paper, "Real-Space Grid Integrals", Eq. 1-5): loop over grid points,
 * enumerate the neighbouring atom images of the point, evaluate the orbitals
 * there and accumulate.  Summation order is the only freedom taken.
 */
#include "gint_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXORB 32      /* orbitals per atom: l <= 2, up to 32 */
#define MAXCHAN 16

/* ------------------------------------------------------------------------ */
/* Real solid harmonics S_lm(x) = r^l Y_lm(x/r), l <= 2, m = -l..l.           */
/* Orthonormal Y_lm; m < 0 sin-type, m > 0 cos-type.                          */
/* ------------------------------------------------------------------------ */
static void solid_harmonics(int l, const double x[3], double *s, double (*ds)[3])
{
    const double c0 = 0.28209479177387814;   /* 1/(2 sqrt(pi)) */
    const double c1 = 0.48860251190291992;   /* sqrt(3/(4 pi)) */
    const double c2a = 1.0925484305920792;   /* sqrt(15/pi)/2 */
    const double c2b = 0.31539156525252005;  /* sqrt(5/pi)/4 */
    const double c2c = 0.54627421529603959;  /* sqrt(15/pi)/4 */
    const double X = x[0], Y = x[1], Z = x[2];
    if (l == 0) {
        s[0] = c0;
        if (ds) { ds[0][0] = ds[0][1] = ds[0][2] = 0.0; }
    } else if (l == 1) {
        s[0] = c1 * Y; s[1] = c1 * Z; s[2] = c1 * X;
        if (ds) {
            ds[0][0] = 0; ds[0][1] = c1; ds[0][2] = 0;
            ds[1][0] = 0; ds[1][1] = 0; ds[1][2] = c1;
            ds[2][0] = c1; ds[2][1] = 0; ds[2][2] = 0;
        }
    } else {
        s[0] = c2a * X * Y;
        s[1] = c2a * Y * Z;
        s[2] = c2b * (2.0 * Z * Z - X * X - Y * Y);
        s[3] = c2a * X * Z;
        s[4] = c2c * (X * X - Y * Y);
        if (ds) {
            ds[0][0] = c2a * Y; ds[0][1] = c2a * X; ds[0][2] = 0;
            ds[1][0] = 0; ds[1][1] = c2a * Z; ds[1][2] = c2a * Y;
            ds[2][0] = -2 * c2b * X; ds[2][1] = -2 * c2b * Y; ds[2][2] = 4 * c2b * Z;
            ds[3][0] = c2a * Z; ds[3][1] = 0; ds[3][2] = c2a * X;
            ds[4][0] = 2 * c2c * X; ds[4][1] = -2 * c2c * Y; ds[4][2] = 0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Radial part p(r), p'(r).                                                  */
/* ------------------------------------------------------------------------ */
static void radial_eval(const oracle_system *s, int sp, int ch, double r, double *p, double *dp)
{
    const double rc = s->sp_rcut[sp];
    if (r >= rc) { *p = 0.0; *dp = 0.0; return; }
    if (s->radial_mode == 1) {
        /* analytic: f = exp(-a r^2) chi(r) */
        const double a = s->chan_alpha[ch];
        const double g = exp(-a * r * r);
        double chi = 1.0, dchi = 0.0;
        const double rs = s->sp_rs[sp];
        if (s->sp_cutoff[sp] && r > rs && rc > rs) {
            const double t = (r - rs) / (rc - rs);
            chi = 1.0 - (10.0 * t * t * t - 15.0 * t * t * t * t + 6.0 * t * t * t * t * t);
            dchi = -(30.0 * t * t - 60.0 * t * t * t + 30.0 * t * t * t * t) / (rc - rs);
        }
        *p = g * chi;
        *dp = -2.0 * a * r * g * chi + g * dchi;
        return;
    }
    /* table: cubic Hermite between knots k and k+1 */
    const double dr = s->sp_dr[sp];
    const int nk = s->sp_nknots[sp];
    long k = (long)floor(r / dr);
    if (k > nk - 2) k = nk - 2;
    if (k < 0) k = 0;
    const double t = r / dr - (double)k;
    const double *f = s->tab_f + s->chan_tab_off[ch];
    const double *fp = s->tab_fp + s->chan_tab_off[ch];
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t;
    const double h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
    *p = h00 * f[k] + h10 * dr * fp[k] + h01 * f[k + 1] + h11 * dr * fp[k + 1];
    const double d00 = 6 * t2 - 6 * t, d10 = 3 * t2 - 4 * t + 1;
    const double d01 = -6 * t2 + 6 * t, d11 = 3 * t2 - 2 * t;
    *dp = (d00 * f[k] + d01 * f[k + 1]) / dr + d10 * fp[k] + d11 * fp[k + 1];
}

static int species_norb(const oracle_system *s, int sp)
{
    int n = 0;
    for (int c = s->sp_chan_off[sp]; c < s->sp_chan_off[sp + 1]; ++c) n += 2 * s->chan_l[c] + 1;
    return n;
}

/* phi_mu(x) and grad phi_mu(x) for all orbitals of a species.
 * grad phi = (p'(r)/r) x S + p grad S; the first term is 0 at r = 0. */
static void orbitals_at(const oracle_system *s, int sp, const double x[3], double *phi, double (*grad)[3])
{
    const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    int mu = 0;
    for (int c = s->sp_chan_off[sp]; c < s->sp_chan_off[sp + 1]; ++c) {
        const int l = s->chan_l[c];
        double p, dp;
        radial_eval(s, sp, c, r, &p, &dp);
        double sh[5], dsh[5][3];
        solid_harmonics(l, x, sh, grad ? dsh : NULL);
        const double q = (r > 0.0) ? dp / r : 0.0;
        for (int m = 0; m < 2 * l + 1; ++m, ++mu) {
            phi[mu] = p * sh[m];
            if (grad)
                for (int a = 0; a < 3; ++a) grad[mu][a] = q * x[a] * sh[m] + p * dsh[m][a];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Block lookup (I, J, R) -> block index: open addressing hash table.        */
/* ------------------------------------------------------------------------ */
typedef struct { int *keys; int *vals; long cap; } bhash;   /* keys: 5 ints per slot, keys[5q] = -1 if empty */

static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t bhash_of(int i, int j, const int r[3])
{
    uint64_t h = mix64((uint64_t)(uint32_t)i);
    h = mix64(h ^ (uint64_t)(uint32_t)j);
    h = mix64(h ^ (uint64_t)(uint32_t)r[0]);
    h = mix64(h ^ (uint64_t)(uint32_t)r[1]);
    return mix64(h ^ (uint64_t)(uint32_t)r[2]);
}

static int bkey_eq(const int *k, int i, int j, const int r[3])
{
    return k[0] == i && k[1] == j && k[2] == r[0] && k[3] == r[1] && k[4] == r[2];
}

static int bhash_build(bhash *hb, const oracle_system *s)
{
    long cap = 16;
    while (cap < 2L * s->nblk + 16) cap <<= 1;
    hb->cap = cap;
    hb->keys = (int *)malloc(sizeof(int) * 5 * cap);
    hb->vals = (int *)malloc(sizeof(int) * cap);
    if (!hb->keys || !hb->vals) return ORACLE_ENOMEM;
    for (long q = 0; q < cap; ++q) hb->keys[5 * q] = -1;
    for (int b = 0; b < s->nblk; ++b) {
        const int i = s->blk_i[b], j = s->blk_j[b];
        const int *r = s->blk_r + 3 * b;
        if (i < 0 || j < 0 || i >= s->natom || j >= s->natom) return ORACLE_EINVAL;
        long q = (long)(bhash_of(i, j, r) & (uint64_t)(cap - 1));
        while (hb->keys[5 * q] != -1 && !bkey_eq(hb->keys + 5 * q, i, j, r)) q = (q + 1) & (cap - 1);
        if (hb->keys[5 * q] != -1) return ORACLE_EINVAL;   /* duplicate block */
        int *k = hb->keys + 5 * q;
        k[0] = i; k[1] = j; k[2] = r[0]; k[3] = r[1]; k[4] = r[2];
        hb->vals[q] = b;
    }
    return ORACLE_OK;
}

static int bhash_find(const bhash *hb, int i, int j, const int r[3])
{
    long q = (long)(bhash_of(i, j, r) & (uint64_t)(hb->cap - 1));
    while (hb->keys[5 * q] != -1) {
        if (bkey_eq(hb->keys + 5 * q, i, j, r)) return hb->vals[q];
        q = (q + 1) & (hb->cap - 1);
    }
    return -1;
}

static void bhash_free(bhash *hb) { free(hb->keys); free(hb->vals); }

/* ------------------------------------------------------------------------ */
/* Neighbour enumeration with a bin list: grid points are binned into         */
/* blocks of grid cells; each bin keeps every (atom, T) whose sphere can      */
/* reach some point of the bin.  The exact test |x| < rcut is applied per     */
/* point, so the resulting set C(g) is exactly the definition's.              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int atom;
    int T[3];
} cand_t;

typedef struct {
    double cell[9], inv[9];   /* inv: frac = x . inv */
    double spacing[3];        /* interplanar spacings */
    int N[3];
    long ng;
    double omega, w;
    int bs[3], M[3];          /* bin size (grid points), bin counts */
    long *bin_ptr;            /* all bins built up front (NULL in the lazy form) */
    cand_t *cand;
    cand_t **lazy;            /* lazy form: candidates of bin b, built on request */
    int *lazy_n;
    int *norb;                /* per atom */
    long *orb_start;          /* unused placeholder for clarity */
    bhash hb;
    int maxcand;
} ctx_t;

static void inv3(const double *a, double *b, double *det)
{
    double d = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) + a[2] * (a[3] * a[7] - a[4] * a[6]);
    *det = d;
    b[0] = (a[4] * a[8] - a[5] * a[7]) / d; b[1] = (a[2] * a[7] - a[1] * a[8]) / d; b[2] = (a[1] * a[5] - a[2] * a[4]) / d;
    b[3] = (a[5] * a[6] - a[3] * a[8]) / d; b[4] = (a[0] * a[8] - a[2] * a[6]) / d; b[5] = (a[2] * a[3] - a[0] * a[5]) / d;
    b[6] = (a[3] * a[7] - a[4] * a[6]) / d; b[7] = (a[1] * a[6] - a[0] * a[7]) / d; b[8] = (a[0] * a[4] - a[1] * a[3]) / d;
}

/* Cartesian position of the (possibly unwrapped) grid index n. */
static void grid_point(const ctx_t *c, const long n[3], double r[3])
{
    const double f0 = (double)n[0] / c->N[0], f1 = (double)n[1] / c->N[1], f2 = (double)n[2] / c->N[2];
    for (int a = 0; a < 3; ++a) r[a] = f0 * c->cell[a] + f1 * c->cell[3 + a] + f2 * c->cell[6 + a];
}

static void ctx_free(ctx_t *c)
{
    free(c->bin_ptr); free(c->cand); free(c->norb);
    if (c->lazy) {
        const long nbin = (long)c->M[0] * c->M[1] * c->M[2];
        for (long b = 0; b < nbin; ++b) free(c->lazy[b]);
        free(c->lazy); free(c->lazy_n);
    }
    bhash_free(&c->hb);
}

/* Candidate atom images of bin b: every (atom, T) whose cutoff sphere can
 * reach a point of the bin (centre distance < rcut + bin radius).  Appends
 * to *buf (capacity *cap, grown as needed); returns the new count. */
static long bin_candidates(const ctx_t *c, const oracle_system *s, long b, cand_t **buf, long *cap, long nc)
{
    const int b0 = (int)(b / ((long)c->M[1] * c->M[2])), b1 = (int)((b / c->M[2]) % c->M[1]), b2 = (int)(b % c->M[2]);
    const long lo[3] = {(long)b0 * c->bs[0], (long)b1 * c->bs[1], (long)b2 * c->bs[2]};
    long hi[3];
    for (int a = 0; a < 3; ++a) {
        hi[a] = lo[a] + c->bs[a] - 1;
        if (hi[a] > c->N[a] - 1) hi[a] = c->N[a] - 1;
    }
    /* bin centre and radius (max distance to its corner points) */
    double ctr[3], rad = 0.0;
    {
        double fl[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
        for (int a = 0; a < 3; ++a)
            ctr[a] = fl[0] / c->N[0] * c->cell[a] + fl[1] / c->N[1] * c->cell[3 + a] + fl[2] / c->N[2] * c->cell[6 + a];
        for (int q = 0; q < 8; ++q) {
            long n[3] = {(q & 1) ? hi[0] : lo[0], (q & 2) ? hi[1] : lo[1], (q & 4) ? hi[2] : lo[2]};
            double r[3];
            grid_point(c, n, r);
            double d2 = 0;
            for (int a = 0; a < 3; ++a) d2 += (r[a] - ctr[a]) * (r[a] - ctr[a]);
            if (sqrt(d2) > rad) rad = sqrt(d2);
        }
        rad += 1e-9;
    }
    for (int i = 0; i < s->natom; ++i) {
        const double reach = s->sp_rcut[s->species[i]] + rad;
        double dx[3];
        for (int a = 0; a < 3; ++a) dx[a] = ctr[a] - s->pos[3 * i + a];
        double u[3];
        for (int a = 0; a < 3; ++a) u[a] = dx[0] * c->inv[a] + dx[1] * c->inv[3 + a] + dx[2] * c->inv[6 + a];
        int tlo[3], thi[3];
        for (int a = 0; a < 3; ++a) {
            tlo[a] = (int)floor(u[a] - reach / c->spacing[a]) - 1;
            thi[a] = (int)ceil(u[a] + reach / c->spacing[a]) + 1;
        }
        for (int t0 = tlo[0]; t0 <= thi[0]; ++t0)
            for (int t1 = tlo[1]; t1 <= thi[1]; ++t1)
                for (int t2 = tlo[2]; t2 <= thi[2]; ++t2) {
                    double d2 = 0;
                    for (int a = 0; a < 3; ++a) {
                        double x = dx[a] - (t0 * c->cell[a] + t1 * c->cell[3 + a] + t2 * c->cell[6 + a]);
                        d2 += x * x;
                    }
                    if (d2 < reach * reach) {
                        if (nc == *cap) {
                            *cap *= 2;
                            *buf = (cand_t *)realloc(*buf, sizeof(cand_t) * (*cap));
                        }
                        (*buf)[nc].atom = i;
                        (*buf)[nc].T[0] = t0; (*buf)[nc].T[1] = t1; (*buf)[nc].T[2] = t2;
                        ++nc;
                    }
                }
    }
    return nc;
}

static int ctx_init(ctx_t *c, const oracle_system *s, int lazy)
{
    memset(c, 0, sizeof(*c));
    if (s->natom < 0 || !s->cell || !s->grid) return ORACLE_EINVAL;
    for (int q = 0; q < 9; ++q) c->cell[q] = s->cell[q];
    double det;
    inv3(c->cell, c->inv, &det);
    if (!(fabs(det) > 0)) return ORACLE_EINVAL;
    c->omega = fabs(det);
    for (int a = 0; a < 3; ++a) {
        /* spacing between lattice planes normal to reciprocal vector a: 1/|b_a|, b_a = column a of inv */
        double bx = c->inv[0 + a], by = c->inv[3 + a], bz = c->inv[6 + a];
        c->spacing[a] = 1.0 / sqrt(bx * bx + by * by + bz * bz);
        c->N[a] = s->grid[a];
        if (c->N[a] <= 0) return ORACLE_EINVAL;
    }
    c->ng = (long)c->N[0] * c->N[1] * c->N[2];
    c->w = c->omega / (double)c->ng;
    c->norb = (int *)malloc(sizeof(int) * (s->natom > 0 ? s->natom : 1));
    for (int i = 0; i < s->natom; ++i) {
        c->norb[i] = species_norb(s, s->species[i]);
        if (c->norb[i] > MAXORB) return ORACLE_EINVAL;
        for (int ch = s->sp_chan_off[s->species[i]]; ch < s->sp_chan_off[s->species[i] + 1]; ++ch)
            if (s->chan_l[ch] < 0 || s->chan_l[ch] > 2) return ORACLE_EINVAL;
    }
    int rc = bhash_build(&c->hb, s);
    if (rc) return rc;
    /* bins of about 8 grid points per axis */
    for (int a = 0; a < 3; ++a) {
        c->bs[a] = c->N[a] < 8 ? c->N[a] : 8;
        c->M[a] = (c->N[a] + c->bs[a] - 1) / c->bs[a];
    }
    const long nbin = (long)c->M[0] * c->M[1] * c->M[2];
    if (lazy) {
        /* bins are built on request (ensure_bins), for callers that visit few points */
        c->lazy = (cand_t **)calloc(nbin, sizeof(cand_t *));
        c->lazy_n = (int *)calloc(nbin, sizeof(int));
        return ORACLE_OK;
    }
    c->bin_ptr = (long *)calloc(nbin + 1, sizeof(long));
    long capc = 1024, nc = 0;
    c->cand = (cand_t *)malloc(sizeof(cand_t) * capc);
    for (long b = 0; b < nbin; ++b) {
        nc = bin_candidates(c, s, b, &c->cand, &capc, nc);
        c->bin_ptr[b + 1] = nc;
        if (nc - c->bin_ptr[b] > c->maxcand) c->maxcand = (int)(nc - c->bin_ptr[b]);
    }
    return ORACLE_OK;
}

/* Bin of the home-cell grid point g. */
static long bin_of(const ctx_t *c, long g)
{
    const long n[3] = {g / ((long)c->N[1] * c->N[2]), (g / c->N[2]) % c->N[1], g % c->N[2]};
    return ((long)(n[0] / c->bs[0]) * c->M[1] + (n[1] / c->bs[1])) * c->M[2] + (n[2] / c->bs[2]);
}

/* Lazy form: build the candidate lists of the bins of points g[0..n). */
static void ensure_bins(ctx_t *c, const oracle_system *s, long n, const long *g)
{
    const long nbin = (long)c->M[0] * c->M[1] * c->M[2];
    unsigned char *want = (unsigned char *)calloc(nbin, 1);
    for (long k = 0; k < n; ++k)
        if (g[k] >= 0 && g[k] < c->ng) want[bin_of(c, g[k])] = 1;
    long nw = 0;
    for (long b = 0; b < nbin; ++b) nw += (want[b] && !c->lazy[b]);
    long *list = (long *)malloc(sizeof(long) * (nw > 0 ? nw : 1));
    nw = 0;
    for (long b = 0; b < nbin; ++b)
        if (want[b] && !c->lazy[b]) list[nw++] = b;
    free(want);
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < nw; ++k) {
        long cap = 64;
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * cap);
        const long cnt = bin_candidates(c, s, list[k], &buf, &cap, 0);
        c->lazy[list[k]] = buf;
        c->lazy_n[list[k]] = (int)cnt;
    }
    for (long k = 0; k < nw; ++k)
        if (c->lazy_n[list[k]] > c->maxcand) c->maxcand = c->lazy_n[list[k]];
    free(list);
}

/* One entry of C(g): atom image and its orbital values/gradients. */
typedef struct {
    int atom, T[3], norb;
    double x[3];
    double phi[MAXORB];
    double grad[MAXORB][3];
} entry_t;

/* Enumerate C(g) for the home-cell grid point g (flat index); fills e[],
 * returns the count.  want_grad selects whether gradients are evaluated. */
static int neighbours(const oracle_system *s, const ctx_t *c, long g, entry_t *e, int want_grad)
{
    const long n[3] = {g / ((long)c->N[1] * c->N[2]), (g / c->N[2]) % c->N[1], g % c->N[2]};
    double r[3];
    grid_point(c, n, r);
    const long b = ((long)(n[0] / c->bs[0]) * c->M[1] + (n[1] / c->bs[1])) * c->M[2] + (n[2] / c->bs[2]);
    const cand_t *cb = c->bin_ptr ? c->cand + c->bin_ptr[b] : c->lazy[b];
    const long nb = c->bin_ptr ? c->bin_ptr[b + 1] - c->bin_ptr[b] : c->lazy_n[b];
    int cnt = 0;
    for (long q = 0; q < nb; ++q) {
        const cand_t *cd = &cb[q];
        const int i = cd->atom, sp = s->species[i];
        double x[3], d2 = 0;
        for (int a = 0; a < 3; ++a) {
            x[a] = r[a] - s->pos[3 * i + a] -
                   (cd->T[0] * c->cell[a] + cd->T[1] * c->cell[3 + a] + cd->T[2] * c->cell[6 + a]);
            d2 += x[a] * x[a];
        }
        const double rc = s->sp_rcut[sp];
        if (!(sqrt(d2) < rc)) continue;
        entry_t *en = &e[cnt++];
        en->atom = i;
        for (int a = 0; a < 3; ++a) { en->T[a] = cd->T[a]; en->x[a] = x[a]; }
        en->norb = c->norb[i];
        orbitals_at(s, sp, x, en->phi, want_grad ? en->grad : NULL);
    }
    return cnt;
}

static int resolve_range(const ctx_t *c, long *g0, long *g1)
{
    if (*g1 < 0 || *g1 > c->ng) *g1 = c->ng;
    if (*g0 < 0) *g0 = 0;
    if (*g0 > *g1) return ORACLE_EINVAL;
    return ORACLE_OK;
}

static int nthreads_max(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* ------------------------------------------------------------------------ */
/* H_IJR (Eq. 2)                                                             */
/* ------------------------------------------------------------------------ */
int oracle_vlocal(const oracle_system *s, const double *v, double *h, long g0, long g1)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 0);
    if (rc) { ctx_free(&c); return rc; }
    if ((rc = resolve_range(&c, &g0, &g1))) { ctx_free(&c); return rc; }
    long nnz = 0;
    for (int b = 0; b < s->nblk; ++b) {
        long e = s->blk_off[b] + (long)c.norb[s->blk_i[b]] * c.norb[s->blk_j[b]];
        if (e > nnz) nnz = e;
    }
    const int nt = nthreads_max();
    double *acc = (double *)calloc((size_t)nt * (nnz > 0 ? nnz : 1), sizeof(double));
    if (!acc) { ctx_free(&c); return ORACLE_ENOMEM; }
    int err = ORACLE_OK;
#pragma omp parallel
    {
        double *hl = acc + (size_t)thread_id() * (nnz > 0 ? nnz : 1);
        entry_t *e = (entry_t *)malloc(sizeof(entry_t) * (c.maxcand + 1));
#pragma omp for schedule(dynamic, 64)
        for (long g = g0; g < g1; ++g) {
            const int n = neighbours(s, &c, g, e, 0);
            const double wv = c.w * v[g];
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    const int R[3] = {e[q].T[0] - e[p].T[0], e[q].T[1] - e[p].T[1], e[q].T[2] - e[p].T[2]};
                    const int blk = bhash_find(&c.hb, e[p].atom, e[q].atom, R);
                    if (blk < 0) {
#pragma omp atomic write
                        err = ORACLE_EPATTERN;
                        continue;
                    }
                    double *hb = hl + s->blk_off[blk];
                    const int nj = e[q].norb;
                    for (int mu = 0; mu < e[p].norb; ++mu) {
                        const double a = wv * e[p].phi[mu];
                        for (int nu = 0; nu < nj; ++nu) hb[mu * nj + nu] += a * e[q].phi[nu];
                    }
                }
        }
        free(e);
    }
    if (err == ORACLE_OK) {
        for (long k = 0; k < nnz; ++k) {
            double sum = 0.0;
            for (int t = 0; t < nt; ++t) sum += acc[(size_t)t * nnz + k];
            h[k] = sum;
        }
    }
    free(acc);
    ctx_free(&c);
    return err;
}

/* D_sym entry for the (I, J, R) block: (D_IJR[mu,nu] + D_JI(-R)[nu,mu]) / 2 */
static int dsym_block(const oracle_system *s, const ctx_t *c, const double *d, int I, int J, const int R[3],
                      double *out /* [nI][nJ] */)
{
    const int b = bhash_find(&c->hb, I, J, R);
    const int Rm[3] = {-R[0], -R[1], -R[2]};
    const int bt = bhash_find(&c->hb, J, I, Rm);
    if (b < 0 || bt < 0) return ORACLE_EPATTERN;
    const int ni = c->norb[I], nj = c->norb[J];
    const double *db = d + s->blk_off[b], *dt = d + s->blk_off[bt];
    for (int mu = 0; mu < ni; ++mu)
        for (int nu = 0; nu < nj; ++nu) out[mu * nj + nu] = 0.5 * (db[mu * nj + nu] + dt[nu * ni + mu]);
    return ORACLE_OK;
}

/* rho_g (Eq. 3) at one point from its neighbour list.  With absval, the sum
 * of the magnitudes of its terms, sum |phi_Imu| |D_IJR[mu,nu]| |phi_Jnu|: the
 * scale that rounding errors of a reordered or lower-precision evaluation of
 * rho_g are proportional to (rho_g itself can be much smaller by cancellation). */
static int rho_at(const oracle_system *s, const ctx_t *c, const double *d, const entry_t *e, int n, int absval,
                  double *out)
{
    double rho = 0.0;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            const int R[3] = {e[q].T[0] - e[p].T[0], e[q].T[1] - e[p].T[1], e[q].T[2] - e[p].T[2]};
            const int blk = bhash_find(&c->hb, e[p].atom, e[q].atom, R);
            if (blk < 0) return ORACLE_EPATTERN;
            const double *db = d + s->blk_off[blk];
            const int nj = e[q].norb;
            for (int mu = 0; mu < e[p].norb; ++mu) {
                double t = 0.0;
                if (absval)
                    for (int nu = 0; nu < nj; ++nu) t += fabs(db[mu * nj + nu]) * fabs(e[q].phi[nu]);
                else
                    for (int nu = 0; nu < nj; ++nu) t += db[mu * nj + nu] * e[q].phi[nu];
                rho += (absval ? fabs(e[p].phi[mu]) : e[p].phi[mu]) * t;
            }
        }
    *out = rho;
    return ORACLE_OK;
}

static int rho_range(const oracle_system *s, const double *d, double *rho, long g0, long g1, int absval)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 0);
    if (rc) { ctx_free(&c); return rc; }
    if ((rc = resolve_range(&c, &g0, &g1))) { ctx_free(&c); return rc; }
    int err = ORACLE_OK;
#pragma omp parallel
    {
        entry_t *e = (entry_t *)malloc(sizeof(entry_t) * (c.maxcand + 1));
#pragma omp for schedule(dynamic, 64)
        for (long g = g0; g < g1; ++g) {
            const int n = neighbours(s, &c, g, e, 0);
            double r;
            if (rho_at(s, &c, d, e, n, absval, &r)) {
#pragma omp atomic write
                err = ORACLE_EPATTERN;
                r = 0.0;
            }
            rho[g] = r;
        }
        free(e);
    }
    ctx_free(&c);
    return err;
}

int oracle_rho(const oracle_system *s, const double *d, double *rho, long g0, long g1)
{
    return rho_range(s, d, rho, g0, g1, 0);
}

int oracle_rho_abs(const oracle_system *s, const double *d, double *out, long g0, long g1)
{
    return rho_range(s, d, out, g0, g1, 1);
}

static int rho_points(const oracle_system *s, const double *d, long npts, const long *gidx, double *out, int absval)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 1);
    if (rc) { ctx_free(&c); return rc; }
    ensure_bins(&c, s, npts, gidx);
    int err = ORACLE_OK;
#pragma omp parallel
    {
        entry_t *e = (entry_t *)malloc(sizeof(entry_t) * (c.maxcand + 1));
#pragma omp for schedule(dynamic, 16)
        for (long k = 0; k < npts; ++k) {
            const long g = gidx[k];
            if (g < 0 || g >= c.ng) {
#pragma omp atomic write
                err = ORACLE_EINVAL;
                continue;
            }
            const int n = neighbours(s, &c, g, e, 0);
            double r;
            if (rho_at(s, &c, d, e, n, absval, &r)) {
#pragma omp atomic write
                err = ORACLE_EPATTERN;
                r = 0.0;
            }
            out[k] = r;
        }
        free(e);
    }
    ctx_free(&c);
    return err;
}

int oracle_rho_points(const oracle_system *s, const double *d, long npts, const long *gidx, double *out)
{
    return rho_points(s, d, npts, gidx, out, 0);
}

int oracle_rho_abs_points(const oracle_system *s, const double *d, long npts, const long *gidx, double *out)
{
    return rho_points(s, d, npts, gidx, out, 1);
}

/* Force/strain contributions of one grid point (Eq. 4 and 5, readings in the
 * header): for every entry p = (K, T, mu) of C(g),
 *   psi_mu = sum_{q = (J,T',nu)} Dsym_(K,J,T'-T)[mu,nu] phi_q,nu
 *   F_K   += 2 w V_g sum_mu grad phi_p,mu psi_mu
 *   Z_ab  += 2 w V_g sum_mu d_a phi_p,mu x_p,b psi_mu
 * and the energy density term w V_g rho_g.  Only entries with atom == only
 * (if only >= 0) contribute to F/Z. */
static int force_at(const oracle_system *s, const ctx_t *c, const double *d, const entry_t *e, int n,
                    double wv, int only, double *F /* [natom][3] or [3] */, double *Z, double *erho)
{
    double dsym[MAXORB * MAXORB];
    double rho = 0.0;
    for (int p = 0; p < n; ++p) {
        double psi[MAXORB];
        for (int mu = 0; mu < e[p].norb; ++mu) psi[mu] = 0.0;
        for (int q = 0; q < n; ++q) {
            const int R[3] = {e[q].T[0] - e[p].T[0], e[q].T[1] - e[p].T[1], e[q].T[2] - e[p].T[2]};
            if (dsym_block(s, c, d, e[p].atom, e[q].atom, R, dsym)) return ORACLE_EPATTERN;
            const int nj = e[q].norb;
            for (int mu = 0; mu < e[p].norb; ++mu) {
                double t = 0.0;
                for (int nu = 0; nu < nj; ++nu) t += dsym[mu * nj + nu] * e[q].phi[nu];
                psi[mu] += t;
            }
        }
        for (int mu = 0; mu < e[p].norb; ++mu) rho += e[p].phi[mu] * psi[mu];
        if (only >= 0 && e[p].atom != only) continue;
        double *Fk = (only >= 0) ? F : F + 3 * e[p].atom;
        for (int mu = 0; mu < e[p].norb; ++mu)
            for (int a = 0; a < 3; ++a) {
                const double t = 2.0 * wv * e[p].grad[mu][a] * psi[mu];
                Fk[a] += t;
                for (int b2 = 0; b2 < 3; ++b2) Z[3 * a + b2] += t * e[p].x[b2];
            }
    }
    *erho = wv * rho;
    return ORACLE_OK;
}

int oracle_force_stress(const oracle_system *s, const double *v, const double *d,
                        double *force, double *zstrain, double *energy, long g0, long g1)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 0);
    if (rc) { ctx_free(&c); return rc; }
    if ((rc = resolve_range(&c, &g0, &g1))) { ctx_free(&c); return rc; }
    const int nt = nthreads_max();
    const int na = s->natom > 0 ? s->natom : 1;
    double *Facc = (double *)calloc((size_t)nt * 3 * na, sizeof(double));
    double *Zacc = (double *)calloc((size_t)nt * 9, sizeof(double));
    double *Eacc = (double *)calloc((size_t)nt, sizeof(double));
    int err = ORACLE_OK;
#pragma omp parallel
    {
        const int t = thread_id();
        entry_t *e = (entry_t *)malloc(sizeof(entry_t) * (c.maxcand + 1));
#pragma omp for schedule(dynamic, 64)
        for (long g = g0; g < g1; ++g) {
            const int n = neighbours(s, &c, g, e, 1);
            double er;
            if (force_at(s, &c, d, e, n, c.w * v[g], -1, Facc + (size_t)t * 3 * na, Zacc + 9 * t, &er)) {
#pragma omp atomic write
                err = ORACLE_EPATTERN;
                continue;
            }
            Eacc[t] += er;
        }
        free(e);
    }
    if (err == ORACLE_OK) {
        for (int k = 0; k < 3 * s->natom; ++k) {
            double sum = 0.0;
            for (int t = 0; t < nt; ++t) sum += Facc[(size_t)t * 3 * na + k];
            force[k] = sum;
        }
        for (int k = 0; k < 9; ++k) {
            double sum = 0.0;
            for (int t = 0; t < nt; ++t) sum += Zacc[9 * t + k];
            zstrain[k] = sum;
        }
        double es = 0.0;
        for (int t = 0; t < nt; ++t) es += Eacc[t];
        if (energy) *energy = es;
    }
    free(Facc); free(Zacc); free(Eacc);
    ctx_free(&c);
    return err;
}

/* Integer grid-index box enclosing a sphere (centre x0, radius rad). */
static void sphere_box(const ctx_t *c, const double x0[3], double rad, long lo[3], long hi[3])
{
    for (int a = 0; a < 3; ++a) {
        const double u = x0[0] * c->inv[a] + x0[1] * c->inv[3 + a] + x0[2] * c->inv[6 + a];
        const double ext = rad / c->spacing[a];
        lo[a] = (long)floor((u - ext) * c->N[a]) - 1;
        hi[a] = (long)ceil((u + ext) * c->N[a]) + 1;
    }
}

static long floordiv(long a, long b) { long q = a / b; if ((a % b != 0) && ((a < 0) != (b < 0))) --q; return q; }

/* H for selected blocks: the same sum written over the unwrapped grid
 * points n (r_n = r_g + T0.h), H_IJR = sum_n w V_{n mod N} phi_I(r_n - tau_I)
 * phi_J(r_n - tau_J - R.h). */
int oracle_vlocal_blocks(const oracle_system *s, const double *v, int nsel, const int *blk, double *out)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 1);
    if (rc) { ctx_free(&c); return rc; }
    long *outoff = (long *)malloc(sizeof(long) * (nsel + 1));
    outoff[0] = 0;
    for (int k = 0; k < nsel; ++k) {
        if (blk[k] < 0 || blk[k] >= s->nblk) { free(outoff); ctx_free(&c); return ORACLE_EINVAL; }
        outoff[k + 1] = outoff[k] + (long)c.norb[s->blk_i[blk[k]]] * c.norb[s->blk_j[blk[k]]];
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < nsel; ++k) {
        const int b = blk[k], I = s->blk_i[b], J = s->blk_j[b];
        const int *R = s->blk_r + 3 * b;
        const int ni = c.norb[I], nj = c.norb[J];
        double *o = out + outoff[k];
        for (int q = 0; q < ni * nj; ++q) o[q] = 0.0;
        double tJ[3];
        for (int a = 0; a < 3; ++a)
            tJ[a] = s->pos[3 * J + a] + R[0] * c.cell[a] + R[1] * c.cell[3 + a] + R[2] * c.cell[6 + a];
        const double rcI = s->sp_rcut[s->species[I]], rcJ = s->sp_rcut[s->species[J]];
        long lo[3], hi[3];
        sphere_box(&c, s->pos + 3 * I, rcI, lo, hi);
        double phi_i[MAXORB], phi_j[MAXORB];
        for (long n0 = lo[0]; n0 <= hi[0]; ++n0)
            for (long n1 = lo[1]; n1 <= hi[1]; ++n1)
                for (long n2 = lo[2]; n2 <= hi[2]; ++n2) {
                    const long n[3] = {n0, n1, n2};
                    double r[3], xi[3], xj[3], di = 0, dj = 0;
                    grid_point(&c, n, r);
                    for (int a = 0; a < 3; ++a) {
                        xi[a] = r[a] - s->pos[3 * I + a]; di += xi[a] * xi[a];
                        xj[a] = r[a] - tJ[a]; dj += xj[a] * xj[a];
                    }
                    if (!(sqrt(di) < rcI) || !(sqrt(dj) < rcJ)) continue;
                    const long g = ((n0 - floordiv(n0, c.N[0]) * c.N[0]) * c.N[1] + (n1 - floordiv(n1, c.N[1]) * c.N[1])) * c.N[2] +
                                   (n2 - floordiv(n2, c.N[2]) * c.N[2]);
                    orbitals_at(s, s->species[I], xi, phi_i, NULL);
                    orbitals_at(s, s->species[J], xj, phi_j, NULL);
                    const double wv = c.w * v[g];
                    for (int mu = 0; mu < ni; ++mu)
                        for (int nu = 0; nu < nj; ++nu) o[mu * nj + nu] += wv * phi_i[mu] * phi_j[nu];
                }
    }
    free(outoff);
    ctx_free(&c);
    return ORACLE_OK;
}

/* Force and strain contribution of selected atoms K: the sum over grid
 * points restricted to entries of C(g) that belong to atom K. */
int oracle_force_atoms(const oracle_system *s, const double *v, const double *d,
                       int nsel, const int *atoms, double *force, double *zstrain)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 1);
    if (rc) { ctx_free(&c); return rc; }
    int err = ORACLE_OK;
    for (int k = 0; k < nsel; ++k)
        if (atoms[k] < 0 || atoms[k] >= s->natom) { ctx_free(&c); return ORACLE_EINVAL; }
    for (int k = 0; k < nsel; ++k) {
        const int K = atoms[k];
        const double rcK = s->sp_rcut[s->species[K]];
        long lo[3], hi[3];
        sphere_box(&c, s->pos + 3 * K, rcK, lo, hi);
        const int nt = nthreads_max();
        double *Fa = (double *)calloc((size_t)nt * 3, sizeof(double));
        double *Za = (double *)calloc((size_t)nt * 9, sizeof(double));
        /* Collect the home-cell points whose neighbour set holds an image of K:
         * every unwrapped point n of K's sphere maps to g = n mod N. */
        const long nb0 = hi[0] - lo[0] + 1, nb1 = hi[1] - lo[1] + 1, nb2 = hi[2] - lo[2] + 1;
        const long tot = nb0 * nb1 * nb2;
        unsigned char *seen = (unsigned char *)calloc((size_t)c.ng, 1);
        for (long q = 0; q < tot; ++q) {
            const long n[3] = {lo[0] + q / (nb1 * nb2), lo[1] + (q / nb2) % nb1, lo[2] + q % nb2};
            double r[3], d2 = 0;
            grid_point(&c, n, r);
            for (int a = 0; a < 3; ++a) d2 += (r[a] - s->pos[3 * K + a]) * (r[a] - s->pos[3 * K + a]);
            if (!(sqrt(d2) < rcK)) continue;
            const long g = ((n[0] - floordiv(n[0], c.N[0]) * c.N[0]) * c.N[1] + (n[1] - floordiv(n[1], c.N[1]) * c.N[1])) * c.N[2] +
                           (n[2] - floordiv(n[2], c.N[2]) * c.N[2]);
            seen[g] = 1;
        }
        long npt = 0;
        for (long g = 0; g < c.ng; ++g) npt += seen[g];
        long *pts = (long *)malloc(sizeof(long) * (npt > 0 ? npt : 1));
        npt = 0;
        for (long g = 0; g < c.ng; ++g)
            if (seen[g]) pts[npt++] = g;
        free(seen);
        ensure_bins(&c, s, npt, pts);
#pragma omp parallel
        {
            const int t = thread_id();
            entry_t *e = (entry_t *)malloc(sizeof(entry_t) * (c.maxcand + 1));
#pragma omp for schedule(dynamic, 64)
            for (long q = 0; q < npt; ++q) {
                const long g = pts[q];
                const int n = neighbours(s, &c, g, e, 1);
                double er;
                if (force_at(s, &c, d, e, n, c.w * v[g], K, Fa + 3 * t, Za + 9 * t, &er)) {
#pragma omp atomic write
                    err = ORACLE_EPATTERN;
                }
            }
            free(e);
        }
        for (int a = 0; a < 3; ++a) {
            double sum = 0;
            for (int t = 0; t < nt; ++t) sum += Fa[3 * t + a];
            force[3 * k + a] = sum;
        }
        for (int a = 0; a < 9; ++a) {
            double sum = 0;
            for (int t = 0; t < nt; ++t) sum += Za[9 * t + a];
            if (zstrain) zstrain[9 * k + a] = sum;
        }
        free(Fa); free(Za); free(pts);
    }
    ctx_free(&c);
    return err;
}

int oracle_orbitals(const oracle_system *s, int sp, long n, const double *x, double *phi, double *grad)
{
    if (sp < 0 || sp >= s->nspecies) return ORACLE_EINVAL;
    const int no = species_norb(s, sp);
    if (no > MAXORB) return ORACLE_EINVAL;
    for (long k = 0; k < n; ++k) {
        double ph[MAXORB], gr[MAXORB][3];
        const double *xk = x + 3 * k;
        const double r = sqrt(xk[0] * xk[0] + xk[1] * xk[1] + xk[2] * xk[2]);
        if (!(r < s->sp_rcut[sp])) {
            for (int m = 0; m < no; ++m) { ph[m] = 0; gr[m][0] = gr[m][1] = gr[m][2] = 0; }
        } else {
            orbitals_at(s, sp, xk, ph, gr);
        }
        for (int m = 0; m < no; ++m) {
            phi[k * no + m] = ph[m];
            if (grad) for (int a = 0; a < 3; ++a) grad[(k * no + m) * 3 + a] = gr[m][a];
        }
    }
    return ORACLE_OK;
}

int oracle_radial(const oracle_system *s, int sp, int chan, long n, const double *r, double *p, double *dp)
{
    if (sp < 0 || sp >= s->nspecies) return ORACLE_EINVAL;
    const int ch = s->sp_chan_off[sp] + chan;
    if (chan < 0 || ch >= s->sp_chan_off[sp + 1]) return ORACLE_EINVAL;
    for (long k = 0; k < n; ++k) radial_eval(s, sp, ch, r[k], &p[k], &dp[k]);
    return ORACLE_OK;
}

int oracle_neighbours(const oracle_system *s, long g, int cap, int *atom, int *T, double *x)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 1);
    if (rc) { ctx_free(&c); return rc; }
    if (g < 0 || g >= c.ng) { ctx_free(&c); return ORACLE_EINVAL; }
    ensure_bins(&c, s, 1, &g);
    entry_t *e = (entry_t *)malloc(sizeof(entry_t) * (c.maxcand + 1));
    const int n = neighbours(s, &c, g, e, 0);
    for (int k = 0; k < n && k < cap; ++k) {
        atom[k] = e[k].atom;
        for (int a = 0; a < 3; ++a) { T[3 * k + a] = e[k].T[a]; x[3 * k + a] = e[k].x[a]; }
    }
    free(e);
    ctx_free(&c);
    return n;
}

int oracle_work(const oracle_system *s, long g0, long g1, double *w_out)
{
    ctx_t c;
    int rc = ctx_init(&c, s, 0);
    if (rc) { ctx_free(&c); return rc; }
    if ((rc = resolve_range(&c, &g0, &g1))) { ctx_free(&c); return rc; }
    double W = 0.0;
#pragma omp parallel reduction(+ : W)
    {
        entry_t *e = (entry_t *)malloc(sizeof(entry_t) * (c.maxcand + 1));
        (void)e;
#pragma omp for schedule(dynamic, 256)
        for (long g = g0; g < g1; ++g) {
            /* count orbitals of C(g) without evaluating them */
            const long n[3] = {g / ((long)c.N[1] * c.N[2]), (g / c.N[2]) % c.N[1], g % c.N[2]};
            double r[3];
            grid_point(&c, n, r);
            const long b = ((long)(n[0] / c.bs[0]) * c.M[1] + (n[1] / c.bs[1])) * c.M[2] + (n[2] / c.bs[2]);
            double no = 0;
            for (long q = c.bin_ptr[b]; q < c.bin_ptr[b + 1]; ++q) {
                const cand_t *cd = &c.cand[q];
                const int i = cd->atom;
                double d2 = 0;
                for (int a = 0; a < 3; ++a) {
                    double x = r[a] - s->pos[3 * i + a] -
                               (cd->T[0] * c.cell[a] + cd->T[1] * c.cell[3 + a] + cd->T[2] * c.cell[6 + a]);
                    d2 += x * x;
                }
                if (sqrt(d2) < s->sp_rcut[s->species[i]]) no += c.norb[i];
            }
            W += no * no;
        }
        free(e);
    }
    *w_out = W;
    ctx_free(&c);
    return ORACLE_OK;
}

int oracle_num_threads(void) { return nthreads_max(); }

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
