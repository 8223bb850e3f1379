/* Runs the FP64 oracle on a system dumped by tests/test_sanitizers.py, as a
 * standalone program, so that it can be built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (no Python in the process).  Reads the arrays
 * of <dir>/ (raw little-endian files, sizes in meta.txt), runs Vlocal, rho,
 * force/stress, rho_abs and the work count over all grid points, and writes
 * h, rho, force, zstrain, energy, rho_abs and work back into <dir>/.
 * Test infrastructure only. */
#include <stdio.h>
#include <stdlib.h>

#include "gint_oracle.h"

static void *load(const char *dir, const char *name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(2);
    }
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read %s\n", path);
        exit(2);
    }
    fclose(f);
    return p;
}

static void save(const char *dir, const char *name, const void *p, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fclose(f);
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s <dir>\n", argv[0]);
        return 2;
    }
    const char *dir = argv[1];
    long natom, nspecies, nblk, ngrid, nnz, nchan, knots, mode;
    {
        char path[4096];
        snprintf(path, sizeof path, "%s/meta.txt", dir);
        FILE *f = fopen(path, "r");
        if (!f || fscanf(f, "%ld %ld %ld %ld %ld %ld %ld %ld", &natom, &nspecies, &nblk, &ngrid, &nnz, &nchan,
                         &knots, &mode) != 8) {
            fprintf(stderr, "bad meta.txt\n");
            return 2;
        }
        fclose(f);
    }
    oracle_system s;
    s.natom = (int)natom;
    s.cell = load(dir, "cell.f64", 9 * sizeof(double));
    s.pos = load(dir, "pos.f64", (size_t)natom * 3 * sizeof(double));
    s.species = load(dir, "species.i32", (size_t)natom * sizeof(int));
    s.nspecies = (int)nspecies;
    s.sp_rcut = load(dir, "sp_rcut.f64", (size_t)nspecies * sizeof(double));
    s.sp_dr = load(dir, "sp_dr.f64", (size_t)nspecies * sizeof(double));
    s.sp_rs = load(dir, "sp_rs.f64", (size_t)nspecies * sizeof(double));
    s.sp_nknots = load(dir, "sp_nknots.i32", (size_t)nspecies * sizeof(int));
    s.sp_cutoff = load(dir, "sp_cutoff.i32", (size_t)nspecies * sizeof(int));
    s.sp_chan_off = load(dir, "sp_chan_off.i32", (size_t)(nspecies + 1) * sizeof(int));
    s.chan_l = load(dir, "chan_l.i32", (size_t)nchan * sizeof(int));
    s.chan_alpha = load(dir, "chan_alpha.f64", (size_t)nchan * sizeof(double));
    s.chan_tab_off = load(dir, "chan_tab_off.i64", (size_t)nchan * sizeof(long));
    s.tab_f = load(dir, "tab_f.f64", (size_t)knots * sizeof(double));
    s.tab_fp = load(dir, "tab_fp.f64", (size_t)knots * sizeof(double));
    s.grid = load(dir, "grid.i32", 3 * sizeof(int));
    s.nblk = (int)nblk;
    s.blk_i = load(dir, "blk_i.i32", (size_t)nblk * sizeof(int));
    s.blk_j = load(dir, "blk_j.i32", (size_t)nblk * sizeof(int));
    s.blk_r = load(dir, "blk_r.i32", (size_t)nblk * 3 * sizeof(int));
    s.blk_off = load(dir, "blk_off.i64", (size_t)nblk * sizeof(long));
    s.radial_mode = (int)mode;
    const double *v = load(dir, "v.f64", (size_t)ngrid * sizeof(double));
    const double *d = load(dir, "d.f64", (size_t)nnz * sizeof(double));

    double *h = malloc((size_t)nnz * sizeof(double));
    double *rho = malloc((size_t)ngrid * sizeof(double));
    double *rabs = malloc((size_t)ngrid * sizeof(double));
    double *force = malloc((size_t)natom * 3 * sizeof(double));
    double z[9], e, wk;
    int rc = oracle_vlocal(&s, v, h, 0, -1);
    if (!rc) rc = oracle_rho(&s, d, rho, 0, -1);
    if (!rc) rc = oracle_force_stress(&s, v, d, force, z, &e, 0, -1);
    if (!rc) rc = oracle_rho_abs(&s, d, rabs, 0, -1);
    if (!rc) rc = oracle_work(&s, 0, -1, &wk);
    if (rc) {
        fprintf(stderr, "oracle error %d\n", rc);
        return 1;
    }
    save(dir, "out_h.f64", h, (size_t)nnz * sizeof(double));
    save(dir, "out_rho.f64", rho, (size_t)ngrid * sizeof(double));
    save(dir, "out_rho_abs.f64", rabs, (size_t)ngrid * sizeof(double));
    save(dir, "out_force.f64", force, (size_t)natom * 3 * sizeof(double));
    save(dir, "out_z.f64", z, sizeof z);
    save(dir, "out_e.f64", &e, sizeof e);
    save(dir, "out_work.f64", &wk, sizeof wk);
    free(h);
    free(rho);
    free(rabs);
    free(force);
    free((void *)v);
    free((void *)d);
    free((void *)s.cell);
    free((void *)s.pos);
    free((void *)s.species);
    free((void *)s.sp_rcut);
    free((void *)s.sp_dr);
    free((void *)s.sp_rs);
    free((void *)s.sp_nknots);
    free((void *)s.sp_cutoff);
    free((void *)s.sp_chan_off);
    free((void *)s.chan_l);
    free((void *)s.chan_alpha);
    free((void *)s.chan_tab_off);
    free((void *)s.tab_f);
    free((void *)s.tab_fp);
    free((void *)s.grid);
    free((void *)s.blk_i);
    free((void *)s.blk_j);
    free((void *)s.blk_r);
    free((void *)s.blk_off);
    printf("oracle driver ok: E = %.17g, W = %.17g\n", e, wk);
    return 0;
}
