// Builds the host plan (paper_2409_09399_amd/csrc/gint_plan.cpp, compiled
// here without HIP) for a system dumped by tests/test_sanitizers.py, so that
// the plan builder runs under AddressSanitizer and UndefinedBehaviorSanitizer,
// and checks it against brute force:
//   - the bigcell-stationary bricks: for sampled grid points, every atom
//     image within rcut of the point must be in the union of the point's
//     brick, and for every two such images the pair table must name the
//     pattern block (I, J, T_J - T_I);
//   - the cluster pairs (clusters of up to 4 or up to 8 atoms): over the
//     canonical pairs, the tiles a Vlocal pass stores (block and, for a
//     non-self pair, its transpose) reach no pattern block twice, and reach
//     every block whose two spheres overlap by more than a grid cell;
//   - with slabs=N, the plans of the N slabs along a1: together they hold
//     every (cluster pair, bigcell) visit and every brick of the whole plan
//     exactly once, each in the slab of its origin, with no work item that
//     stores H exclusively.
// Test infrastructure only.
// Usage: plan_driver <dir> [brick=b0,b1,b2] [cl=N] [slabs=N] [nocheck]
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "gint.h"
#include "gint_plan.hpp"

namespace {

template <class T>
std::vector<T> load(const std::string &dir, const char *name, size_t n) {
    std::vector<T> v(n ? n : 1);
    FILE *f = std::fopen((dir + "/" + name).c_str(), "rb");
    if (!f || std::fread(v.data(), sizeof(T), n, f) != n) {
        std::fprintf(stderr, "cannot read %s\n", name);
        std::exit(2);
    }
    std::fclose(f);
    return v;
}

int fail(const char *what, long a = 0, long b = 0) {
    std::fprintf(stderr, "CHECK FAILED: %s (%ld, %ld)\n", what, a, b);
    return 1;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: %s <dir> [brick=b0,b1,b2] [cl=N] [slabs=N] [nocheck]\n", argv[0]);
        return 2;
    }
    bool check = true;
    int brick_arg[3] = {0, 0, 0}, cl_arg = 0, slabs_arg = 1;
    for (int a = 2; a < argc; ++a) {
        const std::string arg = argv[a];
        if (arg == "nocheck")
            check = false;
        else if (arg.rfind("brick=", 0) == 0)
            std::sscanf(arg.c_str() + 6, "%d,%d,%d", &brick_arg[0], &brick_arg[1], &brick_arg[2]);
        else if (arg.rfind("cl=", 0) == 0)
            cl_arg = std::atoi(arg.c_str() + 3);
        else if (arg.rfind("slabs=", 0) == 0)
            slabs_arg = std::atoi(arg.c_str() + 6);
        else {
            std::fprintf(stderr, "unknown argument %s\n", arg.c_str());
            return 2;
        }
    }
    const std::string dir = argv[1];
    long natom, nspecies, nblk, ngrid, nnz, nchan, knots, mode;
    {
        FILE *f = std::fopen((dir + "/meta.txt").c_str(), "r");
        if (!f || std::fscanf(f, "%ld %ld %ld %ld %ld %ld %ld %ld", &natom, &nspecies, &nblk, &ngrid, &nnz, &nchan,
                              &knots, &mode) != 8)
            return 2;
        std::fclose(f);
    }
    auto cell = load<double>(dir, "cell.f64", 9);
    auto pos = load<double>(dir, "pos.f64", natom * 3);
    auto species = load<int>(dir, "species.i32", natom);
    auto rcut = load<double>(dir, "sp_rcut.f64", nspecies);
    auto dr = load<double>(dir, "sp_dr.f64", nspecies);
    auto nk = load<int>(dir, "sp_nknots.i32", nspecies);
    auto choff = load<int>(dir, "sp_chan_off.i32", nspecies + 1);
    auto chan_l = load<int>(dir, "chan_l.i32", nchan);
    auto tab_off = load<long>(dir, "chan_tab_off.i64", nchan);
    auto tab_f = load<double>(dir, "tab_f.f64", knots);
    auto tab_fp = load<double>(dir, "tab_fp.f64", knots);
    auto grid = load<int>(dir, "grid.i32", 3);
    auto bi = load<int>(dir, "blk_i.i32", nblk);
    auto bj = load<int>(dir, "blk_j.i32", nblk);
    auto br = load<int>(dir, "blk_r.i32", nblk * 3);
    auto boff = load<long>(dir, "blk_off.i64", nblk);

    std::vector<gint_species> sps(nspecies);
    for (long s = 0; s < nspecies; ++s) {
        const int c0 = choff[s];
        sps[s].rcut = rcut[s];
        sps[s].dr = dr[s];
        sps[s].nknots = nk[s];
        sps[s].nchan = choff[s + 1] - c0;
        sps[s].chan_l = chan_l.data() + c0;
        sps[s].f = tab_f.data() + tab_off[c0];
        sps[s].fp = tab_fp.data() + tab_off[c0];
    }
    std::vector<int64_t> off64(boff.begin(), boff.end());
    gint_system sys{};
    for (int k = 0; k < 9; ++k) sys.cell[k] = cell[k];
    sys.natom = (int)natom;
    sys.pos = pos.data();
    sys.species = species.data();
    sys.nspecies = (int)nspecies;
    sys.species_list = sps.data();
    for (int k = 0; k < 3; ++k) sys.grid[k] = grid[k];
    sys.nblk = (int)nblk;
    sys.blk_i = bi.data();
    sys.blk_j = bj.data();
    sys.blk_r = br.data();
    sys.blk_off = off64.data();
    gint_options opt{};
    opt.precision = GINT_MIXED_FP16X3;
    for (int k = 0; k < 3; ++k) opt.brick[k] = brick_arg[k];
    opt.cluster_atoms = cl_arg;
    HostPlan hp;
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = gint_build_host_plan(&sys, 1, &opt, true, hp);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc != GINT_OK) {
        std::fprintf(stderr, "plan error %d: %s\n", rc, hp.error.c_str());
        return 1;
    }
    const int B[3] = {hp.brick[0], hp.brick[1], hp.brick[2]};
    const size_t npairs = hp.pairs.size() + hp.pairs8.size();
    if (!check) {
        std::printf("plan built in %.3f s: %zu pairs (clusters of %d), %zu pair bigcells, %zu items, %zu bricks "
                    "(%d x %d x %d), %zu images, %zu pair-table entries\n",
                    secs, npairs, hp.cluster_atoms, hp.bigcells.size(), hp.items_canon.size(), hp.bricks.size(), B[0],
                    B[1], B[2], hp.uatoms.size(), hp.ptab.size());
        return 0;
    }

    // cluster pairs: stores per pattern block over the canonical pairs
    {
        std::map<long long, int> writes;
        auto visit = [&](const auto &pairs, int CL) {
            for (int p = 0; p < hp.ncanon; ++p) {
                const auto &P = pairs[p];
                for (int ia = 0; ia < CL; ++ia)
                    for (int jb = 0; jb < CL; ++jb) {
                        if (P.a[ia] < 0 || P.b[jb] < 0) continue;
                        if (P.hoff[ia * CL + jb] >= 0) ++writes[P.hoff[ia * CL + jb]];
                        if (!P.self && P.hoff_t[ia * CL + jb] >= 0) ++writes[P.hoff_t[ia * CL + jb]];
                    }
            }
        };
        if (!hp.pairs8.empty()) {
            if ((int)hp.pairs8.size() != hp.ncanon || hp.cluster_atoms <= GINT_CL) return fail("8-atom pair list");
            visit(hp.pairs8, GINT_CL8);
        } else {
            if (hp.cluster_atoms > GINT_CL) return fail("4-atom pair list");
            visit(hp.pairs, GINT_CL);
        }
        double hmax = 0;
        for (int k = 0; k < 3; ++k) {
            const double *c = &cell[3 * k];
            hmax = std::max(hmax, std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) / grid[k]);
        }
        long required = 0;
        for (long b = 0; b < nblk; ++b) {
            const auto it = writes.find(boff[b]);
            const int nw = it == writes.end() ? 0 : it->second;
            if (nw > 1) return fail("a pattern block is stored by two tiles", b, nw);
            double d2 = 0;
            for (int c = 0; c < 3; ++c) {
                const double x = pos[3 * bi[b] + c] -
                                 (pos[3 * bj[b] + c] + br[3 * b] * cell[c] + br[3 * b + 1] * cell[3 + c] +
                                  br[3 * b + 2] * cell[6 + c]);
                d2 += x * x;
            }
            // a lens wider than 3 grid steps contains a grid point
            if (std::sqrt(d2) < rcut[species[bi[b]]] + rcut[species[bj[b]]] - 3.0 * hmax) {
                ++required;
                if (nw != 1) return fail("an overlapping pattern block is not stored", b, nw);
            }
        }
        std::printf("cluster pairs ok: %d canonical pairs (clusters of %d), %zu blocks stored, %ld required; ",
                    hp.ncanon, hp.cluster_atoms, writes.size(), required);
    }

    // slabs: the per-slab plans partition the whole plan's work
    if (slabs_arg > 1) {
        typedef std::tuple<std::string, int, int, int> Visit;
        auto visits = [&](const HostPlan &p, std::map<Visit, int> &out) {
            auto add = [&](const auto &pairs, int CL) {
                for (const GItem &it : p.items_canon) {
                    const auto &P = pairs[it.pair];
                    std::string key;
                    for (int k = 0; k < CL; ++k) key += std::to_string(P.a[k]) + "," + std::to_string(P.b[k]) + ";";
                    char sh[96];
                    std::snprintf(sh, sizeof sh, "%.9f,%.9f,%.9f", P.shiftB[0], P.shiftB[1], P.shiftB[2]);
                    key += sh;
                    for (int b = 0; b < it.bc_count; ++b) {
                        const GBig &o = p.bigcells[it.bc_begin + b];
                        ++out[Visit{key, o.x, o.y, o.z}];
                    }
                }
            };
            if (!p.pairs8.empty())
                add(p.pairs8, GINT_CL8);
            else
                add(p.pairs, GINT_CL);
        };
        std::map<Visit, int> whole, parts;
        visits(hp, whole);
        std::map<std::tuple<int, int, int>, int> bricks_whole, bricks_parts;
        for (const GBrick &b : hp.bricks) ++bricks_whole[{b.o[0], b.o[1], b.o[2]}];
        // the slab builds share one pattern index, as the pipeline's do; built
        // in reverse order so the shared index is made by the last slab
        GintSlabShared *shared = gint_slab_shared_new();
        for (int k = slabs_arg - 1; k >= 0; --k) {
            HostPlan sp;
            GintSlab slab;
            slab.count = slabs_arg;
            slab.index = k;
            slab.shared = shared;
            const int r = gint_build_host_plan(&sys, 1, &opt, true, sp, &slab);
            if (r != GINT_OK) {
                gint_slab_shared_free(shared);
                return fail("slab plan", k, r);
            }
            if ((k == slabs_arg - 1) != !sp.blocks.empty()) {
                gint_slab_shared_free(shared);
                return fail("only the first slab build carries the pattern blocks", k);
            }
            if (sp.nnz != hp.nnz) {
                gint_slab_shared_free(shared);
                return fail("slab nnz", (long)sp.nnz, (long)hp.nnz);
            }
            for (const GItem &it : sp.items_canon)
                if (it.pad) return fail("a slab's work item stores H exclusively", k, it.pair);
            for (const GBig &o : sp.bigcells)
                if (!slab.has(((o.x % grid[0]) + grid[0]) % grid[0], grid[0])) return fail("bigcell outside its slab", k, o.x);
            for (const GBrick &b : sp.bricks) {
                if (!slab.has(b.o[0], grid[0])) return fail("brick outside its slab", k, b.o[0]);
                if (sp.brick[0] == hp.brick[0] && sp.brick[1] == hp.brick[1] && sp.brick[2] == hp.brick[2])
                    ++bricks_parts[{b.o[0], b.o[1], b.o[2]}];
            }
            visits(sp, parts);
        }
        gint_slab_shared_free(shared);
        if (parts != whole)
            return fail("the slabs' cluster-pair visits differ from the whole plan's", (long)parts.size(), (long)whole.size());
        for (const auto &kv : parts)
            if (kv.second != 1) return fail("a visit appears twice");
        if (bricks_parts != bricks_whole)
            return fail("the slabs' bricks differ from the whole plan's", (long)bricks_parts.size(), (long)bricks_whole.size());
        std::printf("slabs ok: %d slabs, %zu visits, %zu bricks; ", slabs_arg, whole.size(), bricks_whole.size());
    }

    // brute-force checks of the bricks on sampled grid points
    std::map<std::tuple<int, int, int>, int> brick_at;
    for (size_t k = 0; k < hp.bricks.size(); ++k)
        brick_at[{hp.bricks[k].o[0], hp.bricks[k].o[1], hp.bricks[k].o[2]}] = (int)k;
    std::map<std::tuple<int, int, int, int, int>, int> blk_at;
    for (long b = 0; b < nblk; ++b) blk_at[{bi[b], bj[b], br[3 * b], br[3 * b + 1], br[3 * b + 2]}] = (int)b;
    // lattice images to try: enough to cover rcut beyond the cell
    double rmax = 0;
    for (long s = 0; s < nspecies; ++s) rmax = std::max(rmax, rcut[s]);
    int tmax[3];
    for (int k = 0; k < 3; ++k) {
        const double len = std::sqrt(cell[3 * k] * cell[3 * k] + cell[3 * k + 1] * cell[3 * k + 1] +
                                     cell[3 * k + 2] * cell[3 * k + 2]);
        tmax[k] = (int)std::ceil(rmax / len * 2.0) + 2;
    }
    long checked = 0, images = 0;
    const long stride = std::max(1L, ngrid / 4000);
    for (long g = 0; g < ngrid; g += stride) {
        const int n0 = (int)(g / ((long)grid[1] * grid[2])), n1 = (int)((g / grid[2]) % grid[1]),
                  n2 = (int)(g % grid[2]);
        double r[3];
        for (int c = 0; c < 3; ++c)
            r[c] = n0 * cell[c] / grid[0] + n1 * cell[3 + c] / grid[1] + n2 * cell[6 + c] / grid[2];
        struct Img {
            int atom, t[3];
            double p[3];
        };
        std::vector<Img> in;
        for (long a = 0; a < natom; ++a)
            for (int t0 = -tmax[0]; t0 <= tmax[0]; ++t0)
                for (int t1 = -tmax[1]; t1 <= tmax[1]; ++t1)
                    for (int t2 = -tmax[2]; t2 <= tmax[2]; ++t2) {
                        Img im{(int)a, {t0, t1, t2}, {0, 0, 0}};
                        double d2 = 0;
                        for (int c = 0; c < 3; ++c) {
                            im.p[c] = pos[3 * a + c] + t0 * cell[c] + t1 * cell[3 + c] + t2 * cell[6 + c];
                            d2 += (r[c] - im.p[c]) * (r[c] - im.p[c]);
                        }
                        const double rc = rcut[species[a]];
                        if (d2 < rc * rc && std::sqrt(d2) < rc) in.push_back(im);
                    }
        const int o[3] = {n0 / (4 * B[0]) * 4 * B[0], n1 / (4 * B[1]) * 4 * B[1], n2 / (4 * B[2]) * 4 * B[2]};
        auto it = brick_at.find({o[0], o[1], o[2]});
        if (it == brick_at.end()) {
            if (!in.empty()) return fail("point reached by an atom has no brick", g, (long)in.size());
            continue;
        }
        const GBrick &bk = hp.bricks[it->second];
        std::vector<int> slot(in.size(), -1);
        for (size_t q = 0; q < in.size(); ++q) {
            for (int u = 0; u < bk.u_count; ++u) {
                const GUAtom &ua = hp.uatoms[bk.u_begin + u];
                if (ua.atom == in[q].atom && std::fabs(ua.x - in[q].p[0]) < 1e-9 && std::fabs(ua.y - in[q].p[1]) < 1e-9 &&
                    std::fabs(ua.z - in[q].p[2]) < 1e-9) {
                    slot[q] = u;
                    break;
                }
            }
            if (slot[q] < 0) return fail("atom image within rcut missing from the brick union", g, in[q].atom);
        }
        for (size_t p = 0; p < in.size(); ++p)
            for (size_t q = 0; q < in.size(); ++q) {
                const int want_it = [&] {
                    auto f = blk_at.find({in[p].atom, in[q].atom, in[q].t[0] - in[p].t[0], in[q].t[1] - in[p].t[1],
                                          in[q].t[2] - in[p].t[2]});
                    return f == blk_at.end() ? -1 : f->second;
                }();
                const int got = hp.ptab[bk.pt_off + (long long)slot[p] * bk.u_count + slot[q]];
                if (want_it < 0) return fail("overlapping pair has no pattern block", g, (long)p);
                if (got != want_it) return fail("pair table names the wrong block", got, want_it);
            }
        ++checked;
        images += (long)in.size();
    }
    std::printf("plan driver ok: %zu pairs, %zu items, %zu bricks (%d x %d x %d), %zu images, %ld points checked "
                "(%ld images)\n",
                npairs, hp.items_ordered.size(), hp.bricks.size(), B[0], B[1], B[2], hp.uatoms.size(), checked,
                images);
    return 0;
}
