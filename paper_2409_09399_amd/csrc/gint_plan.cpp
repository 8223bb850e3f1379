// Host plan builder.  See gint_plan.hpp and gint_internal.h for the layout.
#include "gint_plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <string>
#include <unordered_map>

namespace {

struct Vec3 {
    double x, y, z;
};

inline Vec3 sub(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline Vec3 add(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

struct Geometry {
    double cell[9];
    double inv[9];          // frac = x . inv  (column i of inv is reciprocal vector b_i)
    double spacing[3];      // interplanar spacings
    int N[3];
    Vec3 e[3];              // grid step vectors
    Vec3 a[3];              // lattice vectors
    Vec3 lat(int t0, int t1, int t2) const {
        return {t0 * a[0].x + t1 * a[1].x + t2 * a[2].x, t0 * a[0].y + t1 * a[1].y + t2 * a[2].y,
                t0 * a[0].z + t1 * a[1].z + t2 * a[2].z};
    }
    double frac(Vec3 x, int i) const { return x.x * inv[i] + x.y * inv[3 + i] + x.z * inv[6 + i]; }
    Vec3 point(double n0, double n1, double n2) const {
        return {n0 * e[0].x + n1 * e[1].x + n2 * e[2].x, n0 * e[0].y + n1 * e[1].y + n2 * e[2].y,
                n0 * e[0].z + n1 * e[1].z + n2 * e[2].z};
    }
};

// Bigcell record: unwrapped origin, plus the flat index of the wrapped origin
// when none of the bigcell's points wraps (then the kernels index V and rho
// by adding a fixed per-point offset) and the grid has fewer than 2^31 points;
// -1 sends the kernels to the general wrapped index.
GBig make_bigcell(const int N[3], long long o0, long long o1, long long o2) {
    const long long o[3] = {o0, o1, o2};
    long long wr[3];
    bool wraps = (long long)N[0] * N[1] * N[2] > 0x7fffffffLL;
    for (int k = 0; k < 3; ++k) {
        long long m = o[k] % N[k];
        if (m < 0) m += N[k];
        wr[k] = m;
        if (m + GINT_BC > N[k]) wraps = true;
    }
    const long long flat = (wr[0] * N[1] + wr[1]) * N[2] + wr[2];
    return GBig{(int)o0, (int)o1, (int)o2, wraps ? -1 : (int)flat};
}

bool invert3(const double *a, double *b, double *det) {
    double d = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
               a[2] * (a[3] * a[7] - a[4] * a[6]);
    *det = d;
    if (!(std::fabs(d) > 0.0) || !std::isfinite(d)) return false;
    b[0] = (a[4] * a[8] - a[5] * a[7]) / d; b[1] = (a[2] * a[7] - a[1] * a[8]) / d; b[2] = (a[1] * a[5] - a[2] * a[4]) / d;
    b[3] = (a[5] * a[6] - a[3] * a[8]) / d; b[4] = (a[0] * a[8] - a[2] * a[6]) / d; b[5] = (a[2] * a[3] - a[0] * a[5]) / d;
    b[6] = (a[3] * a[7] - a[4] * a[6]) / d; b[7] = (a[1] * a[6] - a[0] * a[7]) / d; b[8] = (a[0] * a[4] - a[1] * a[3]) / d;
    return true;
}

struct BlockKey {
    int i, j, r0, r1, r2;
    bool operator==(const BlockKey &o) const {
        return i == o.i && j == o.j && r0 == o.r0 && r1 == o.r1 && r2 == o.r2;
    }
};

struct BlockKeyHash {
    size_t operator()(const BlockKey &k) const {
        unsigned long long h = 0x9E3779B97F4A7C15ull;
        const int v[5] = {k.i, k.j, k.r0, k.r1, k.r2};
        for (int x : v) {
            h ^= (unsigned long long)(unsigned)x + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
            h *= 0xBF58476D1CE4E5B9ull;
        }
        return (size_t)(h ^ (h >> 31));
    }
};

// (I, J, R) -> element offset of the block, open addressing with linear
// probing (offsets are >= 0; -1 marks an empty slot).
struct BlockMap {
    struct Slot {
        int i, j, r0, r1, r2;
        long long off;
    };
    std::vector<Slot> t;
    size_t mask = 0;
    void reserve(size_t n) {
        size_t cap = 16;
        while (cap < 2 * n + 16) cap <<= 1;
        t.assign(cap, Slot{0, 0, 0, 0, 0, -1});
        mask = cap - 1;
    }
    // false if the key is already present
    bool insert(const BlockKey &k, long long off) {
        size_t h = BlockKeyHash()(k) & mask;
        while (t[h].off >= 0) {
            const Slot &s = t[h];
            if (s.i == k.i && s.j == k.j && s.r0 == k.r0 && s.r1 == k.r1 && s.r2 == k.r2) return false;
            h = (h + 1) & mask;
        }
        t[h] = Slot{k.i, k.j, k.r0, k.r1, k.r2, off};
        return true;
    }
    long long find(int i, int j, int r0, int r1, int r2) const {
        if (t.empty()) return -1;
        size_t h = BlockKeyHash()(BlockKey{i, j, r0, r1, r2}) & mask;
        for (;;) {
            const Slot &s = t[h];
            if (s.off < 0) return -1;
            if (s.i == i && s.j == j && s.r0 == r0 && s.r1 == r1 && s.r2 == r2) return s.off;
            h = (h + 1) & mask;
        }
    }
};

// Recursive bisection of atoms along the longest extent into groups of at
// most cl atoms; left halves take a multiple of cl atoms so clusters are full.
void bisect(const std::vector<Vec3> &pos, std::vector<int> idx, int cl, std::vector<std::vector<int>> &out) {
    if ((int)idx.size() <= cl) {
        out.push_back(idx);
        return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i : idx) {
        const double c[3] = {pos[i].x, pos[i].y, pos[i].z};
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], c[k]); hi[k] = std::max(hi[k], c[k]); }
    }
    int ax = 0;
    for (int k = 1; k < 3; ++k)
        if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
    std::stable_sort(idx.begin(), idx.end(), [&](int p, int q) {
        const double a = ax == 0 ? pos[p].x : ax == 1 ? pos[p].y : pos[p].z;
        const double b = ax == 0 ? pos[q].x : ax == 1 ? pos[q].y : pos[q].z;
        return a < b;
    });
    const int n = (int)idx.size();
    int nl = ((n + 2 * cl - 1) / (2 * cl)) * cl;
    if (nl >= n) nl = n - 1;
    if (nl < 1) nl = 1;
    bisect(pos, std::vector<int>(idx.begin(), idx.begin() + nl), cl, out);
    bisect(pos, std::vector<int>(idx.begin() + nl, idx.end()), cl, out);
}

struct Cluster {
    std::vector<int> atoms;
    Vec3 c;
    double reach;    // max_a |tau_a - c| + rc_a
};

template <int CL>
struct PairOutT {
    GPairT<CL> pair;
    std::vector<GBig> bcs;
};

// (I, J, R) -> block index: per atom I, its blocks sorted by (J, R), found
// by binary search.  The pair-table loops look up many J for one I in a row,
// so the row (a few KB) stays in cache.
struct BlockIndex {
    struct Ent {
        int j, r0, r1, r2, b;
        bool operator<(const Ent &o) const {
            if (j != o.j) return j < o.j;
            if (r0 != o.r0) return r0 < o.r0;
            if (r1 != o.r1) return r1 < o.r1;
            return r2 < o.r2;
        }
    };
    std::vector<size_t> row;   // natom + 1 offsets into ent
    std::vector<Ent> ent;
    std::vector<int> tr;       // per block: the index of its transpose (J, I, -R), -1 if absent
    void build(int nblk, const int *bi, const int *bj, const int *br) {
        int natom = 0;
        for (int b = 0; b < nblk; ++b) natom = std::max(natom, std::max(bi[b], bj[b]) + 1);
        row.assign((size_t)natom + 1, 0);
        for (int b = 0; b < nblk; ++b) ++row[(size_t)bi[b] + 1];
        for (int i = 0; i < natom; ++i) row[(size_t)i + 1] += row[(size_t)i];
        ent.resize((size_t)nblk);
        std::vector<size_t> at(row.begin(), row.end() - 1);
        for (int b = 0; b < nblk; ++b) ent[at[(size_t)bi[b]]++] = Ent{bj[b], br[3 * b], br[3 * b + 1], br[3 * b + 2], b};
        for (int i = 0; i < natom; ++i) std::sort(ent.begin() + row[(size_t)i], ent.begin() + row[(size_t)i + 1]);
        tr.assign((size_t)nblk, -1);
        for (int b = 0; b < nblk; ++b) tr[(size_t)b] = find(bj[b], bi[b], -br[3 * b], -br[3 * b + 1], -br[3 * b + 2]);
    }
    int find(int i, int j, int r0, int r1, int r2) const {
        if (i < 0 || (size_t)i + 1 >= row.size()) return -1;
        const auto lo = ent.begin() + row[(size_t)i], hi = ent.begin() + row[(size_t)i + 1];
        const Ent key{j, r0, r1, r2, 0};
        const auto it = std::lower_bound(lo, hi, key);
        if (it != hi && it->j == j && it->r0 == r0 && it->r1 == r1 && it->r2 == r2) return it->b;
        return -1;
    }
};

// One (brick, atom image) incidence found by the union enumeration.
struct Incidence {
    int brick, atom, t0, t1, t2;
    bool operator<(const Incidence &o) const {
        if (brick != o.brick) return brick < o.brick;
        if (atom != o.atom) return atom < o.atom;
        if (t0 != o.t0) return t0 < o.t0;
        if (t1 != o.t1) return t1 < o.t1;
        return t2 < o.t2;
    }
};

unsigned worker_count() {
    unsigned nth = std::thread::hardware_concurrency();
    if (nth == 0) nth = 4;
    return std::min(nth, 16u);
}

// Runs f(k) for k in [0, n) on worker threads (dynamic assignment).
template <class F>
void parallel_for(int n, F f) {
    std::atomic<int> next{0};
    auto body = [&]() {
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= n) break;
            f(k);
        }
    };
    const unsigned nth = std::min<unsigned>(worker_count(), (unsigned)std::max(1, n));
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nth; ++t) th.emplace_back(body);
    body();
    for (auto &t : th) t.join();
}

// Bricks of B[0] x B[1] x B[2] bigcells tiling the grid [0, N) of one
// system, the atom images whose sphere (radius rcut) reaches a bigcell of
// each brick (tested against the bigcell's circumscribed sphere, radius Rb),
// and the pair tables.  Bricks no atom reaches (vacuum) are left out: their
// points get rho = 0 from the clear that precedes every rho pass.  Returns
// GINT_OK, or 1 if some brick's union exceeds GINT_UMAX (the caller retries
// with smaller bricks).
int build_bricks(const Geometry &G, const std::vector<Vec3> &pos, const std::vector<double> &rc,
                 const std::vector<int> &spec, const BlockIndex &bidx, const int B[3], double Rb, const GintSlab &slab,
                 HostPlan &hp) {
    const int natom = (int)pos.size();
    int nbk[3];
    for (int k = 0; k < 3; ++k) nbk[k] = (G.N[k] + 4 * B[k] - 1) / (4 * B[k]);
    const long long nbricks_all = (long long)nbk[0] * nbk[1] * nbk[2];
    if (nbricks_all > 0x7fffffffLL) return GINT_EINVAL;
    std::vector<std::vector<Incidence>> found(natom);
    parallel_for(natom, [&](int a) {
        const double ext_r = rc[a] + Rb;
        double u[3], ext[3];
        for (int k = 0; k < 3; ++k) {
            u[k] = G.frac(pos[a], k);
            ext[k] = ext_r / G.spacing[k];
        }
        int tlo[3], thi[3];
        for (int k = 0; k < 3; ++k) {
            tlo[k] = (int)std::floor(-u[k] - ext[k]) - 1;
            thi[k] = (int)std::ceil(1.0 - u[k] + ext[k]) + 1;
        }
        const double R2 = ext_r * ext_r;
        std::vector<Incidence> &out = found[a];
        for (int t0 = tlo[0]; t0 <= thi[0]; ++t0)
            for (int t1 = tlo[1]; t1 <= thi[1]; ++t1)
                for (int t2 = tlo[2]; t2 <= thi[2]; ++t2) {
                    const int t[3] = {t0, t1, t2};
                    const Vec3 p = add(pos[a], G.lat(t0, t1, t2));
                    long long blo[3], bhi[3];
                    bool empty = false;
                    for (int k = 0; k < 3; ++k) {
                        const double uu = u[k] + t[k];
                        long long nlo = (long long)std::floor((uu - ext[k]) * G.N[k]) - 4;
                        long long nhi = (long long)std::ceil((uu + ext[k]) * G.N[k]) + 4;
                        nlo = std::max(nlo, 0LL);
                        nhi = std::min(nhi, (long long)G.N[k] - 1);
                        if (nlo > nhi) { empty = true; break; }
                        blo[k] = nlo / (4 * B[k]);
                        bhi[k] = nhi / (4 * B[k]);
                    }
                    if (empty) continue;
                    for (long long b0 = blo[0]; b0 <= bhi[0]; ++b0) {
                        if (!slab.has((int)(4 * B[0] * b0), G.N[0])) continue;
                        for (long long b1 = blo[1]; b1 <= bhi[1]; ++b1)
                            for (long long b2 = blo[2]; b2 <= bhi[2]; ++b2) {
                                bool hit = false;
                                for (int s0 = 0; s0 < B[0] && !hit; ++s0) {
                                    const long long n0 = 4 * (b0 * B[0] + s0);
                                    if (n0 >= G.N[0]) break;
                                    for (int s1 = 0; s1 < B[1] && !hit; ++s1) {
                                        const long long n1 = 4 * (b1 * B[1] + s1);
                                        if (n1 >= G.N[1]) break;
                                        for (int s2 = 0; s2 < B[2] && !hit; ++s2) {
                                            const long long n2 = 4 * (b2 * B[2] + s2);
                                            if (n2 >= G.N[2]) break;
                                            const Vec3 d = sub(G.point(n0 + 1.5, n1 + 1.5, n2 + 1.5), p);
                                            if (dot(d, d) < R2) hit = true;
                                        }
                                    }
                                }
                                if (hit)
                                    out.push_back(Incidence{(int)((b0 * nbk[1] + b1) * nbk[2] + b2), a, t0, t1, t2});
                            }
                    }
                }
    });
    // group by brick, in (brick, atom, image) order: the incidences arrive
    // atom-major with each atom's images in increasing order, so a stable
    // counting sort by brick gives exactly the sorted order
    std::vector<Incidence> all;
    {
        size_t n = 0;
        for (auto &v : found) n += v.size();
        if (nbricks_all <= (1LL << 26)) {
            std::vector<size_t> at((size_t)nbricks_all + 1, 0);
            for (const auto &v : found)
                for (const Incidence &in : v) ++at[(size_t)in.brick + 1];
            for (long long k = 0; k < nbricks_all; ++k) at[(size_t)k + 1] += at[(size_t)k];
            all.resize(n);
            for (auto &v : found) {
                for (const Incidence &in : v) all[at[(size_t)in.brick]++] = in;
                std::vector<Incidence>().swap(v);
            }
        } else {
            all.reserve(n);
            for (auto &v : found) {
                all.insert(all.end(), v.begin(), v.end());
                std::vector<Incidence>().swap(v);
            }
            std::sort(all.begin(), all.end());
        }
    }
    hp.bricks.clear();
    hp.uatoms.clear();
    std::vector<int> utrip;       // image triple of each union entry (pair-table lookups)
    std::vector<int> uatom_idx;
    hp.uatoms.reserve(all.size());
    utrip.reserve(3 * all.size());
    uatom_idx.reserve(all.size());
    for (size_t k = 0; k < all.size();) {
        size_t e = k;
        while (e < all.size() && all[e].brick == all[k].brick) ++e;
        const int n = (int)(e - k);
        if (n > GINT_UMAX) return 1;
        const int bid = all[k].brick;
        GBrick br{};
        const int b2 = bid % nbk[2], b1 = (bid / nbk[2]) % nbk[1], b0 = bid / (nbk[1] * nbk[2]);
        const int bb[3] = {b0, b1, b2};
        for (int q = 0; q < 3; ++q) {
            br.o[q] = 4 * B[q] * bb[q];
            br.nb[q] = std::min(B[q], (G.N[q] - br.o[q] + 3) / 4);
        }
        br.sys = 0;
        br.u_begin = (int)hp.uatoms.size();
        br.u_count = n;
        for (size_t q = k; q < e; ++q) {
            const Incidence &in = all[q];
            const Vec3 p = add(pos[in.atom], G.lat(in.t0, in.t1, in.t2));
            hp.uatoms.push_back(GUAtom{p.x, p.y, p.z, in.atom, spec[in.atom]});
            utrip.push_back(in.t0);
            utrip.push_back(in.t1);
            utrip.push_back(in.t2);
            uatom_idx.push_back(in.atom);
        }
        hp.bricks.push_back(br);
        k = e;
    }
    long long total = 0;
    for (GBrick &br : hp.bricks) {
        br.pt_off = total;
        total += (long long)br.u_count * br.u_count;
    }
    hp.ptab.resize((size_t)total);   // every entry is written below
    parallel_for((int)hp.bricks.size(), [&](int k) {
        const GBrick &br = hp.bricks[k];
        const int n = br.u_count;
        int *pt = hp.ptab.data() + br.pt_off;
        // (j, i) is the transpose block of (i, j): one lookup per unordered pair
        for (int i = 0; i < n; ++i) {
            const int ui = br.u_begin + i;
            const int *ti = &utrip[3 * (size_t)ui];
            for (int j = i; j < n; ++j) {
                const int uj = br.u_begin + j;
                const int *tj = &utrip[3 * (size_t)uj];
                const int b = bidx.find(uatom_idx[ui], uatom_idx[uj], tj[0] - ti[0], tj[1] - ti[1], tj[2] - ti[2]);
                pt[(size_t)i * n + j] = b;
                if (j != i) pt[(size_t)j * n + i] = b >= 0 ? bidx.tr[(size_t)b] : -1;
            }
        }
    });
    (void)natom;
    return GINT_OK;
}

// Bigcell circumradius: centre at offset 1.5 grid steps, corners at +-1.5
// (slightly enlarged so that rounding never drops a point on the sphere).
double bigcell_radius(const Geometry &G) {
    double Rb = 0;
    for (int q = 0; q < 8; ++q) {
        const Vec3 d = G.point((q & 1) ? 1.5 : -1.5, (q & 2) ? 1.5 : -1.5, (q & 4) ? 1.5 : -1.5);
        Rb = std::max(Rb, std::sqrt(dot(d, d)));
    }
    Rb *= 1.0 + 1e-12;
    Rb += 1e-12;
    return Rb;
}

}  // namespace

struct GintSlabShared {
    bool pattern = false;
    BlockMap bm;
    long long nnz = 0;
    bool index = false;
    BlockIndex bidx;
};

GintSlabShared *gint_slab_shared_new() { return new GintSlabShared(); }
void gint_slab_shared_free(GintSlabShared *s) { delete s; }

// Clusters of at most cl atoms (spatial bisection), the cluster pairs that
// overlap on the grid with their bigcell lists, and the work items over them
// (canonical pairs; with_swapped also adds the swapped copy of every
// non-self pair and the items that cover both orders).
template <int CL>
int build_cluster_pairs(const Geometry &G, const std::vector<Vec3> &pos, const std::vector<double> &rc,
                        const BlockMap &bm, int cl, int maxbc_opt, double Rb, bool with_swapped, const GintSlab &slab,
                        std::vector<GPairT<CL>> &pairs, HostPlan &hp) {
    auto fail = [&](int code, const char *msg) {
        hp.error = msg;
        return code;
    };
    const int natom = (int)pos.size();
    // ---- clusters
    std::vector<std::vector<int>> groups;
    {
        std::vector<int> all(natom);
        for (int i = 0; i < natom; ++i) all[i] = i;
        bisect(pos, all, cl, groups);
    }
    std::vector<Cluster> cls(groups.size());
    for (size_t c = 0; c < groups.size(); ++c) {
        Cluster &C = cls[c];
        C.atoms = groups[c];
        Vec3 m{0, 0, 0};
        for (int a : C.atoms) m = add(m, pos[a]);
        m = {m.x / C.atoms.size(), m.y / C.atoms.size(), m.z / C.atoms.size()};
        C.c = m;
        C.reach = 0;
        for (int a : C.atoms) C.reach = std::max(C.reach, std::sqrt(dot(sub(pos[a], m), sub(pos[a], m))) + rc[a]);
    }
    hp.ncluster = (int)cls.size();

    // ---- cluster pairs: (A, B, T) with A < B, or A == B and T >= 0 lexicographically
    const int ncl = (int)cls.size();
    std::vector<std::vector<PairOutT<CL>>> per_a(ncl);
    std::atomic<int> next{0};
    std::atomic<int> err{GINT_OK};
    auto worker = [&]() {
        for (;;) {
            const int A = next.fetch_add(1);
            if (A >= ncl || err.load() != GINT_OK) break;
            const Cluster &CA = cls[A];
            for (int B = A; B < ncl; ++B) {
                const Cluster &CB = cls[B];
                const Vec3 dc = sub(CA.c, CB.c);
                const double reach = CA.reach + CB.reach;
                int tlo[3], thi[3];
                for (int k = 0; k < 3; ++k) {
                    const double u = G.frac(dc, k);
                    tlo[k] = (int)std::floor(u - reach / G.spacing[k]) - 1;
                    thi[k] = (int)std::ceil(u + reach / G.spacing[k]) + 1;
                }
                for (int t0 = tlo[0]; t0 <= thi[0]; ++t0)
                    for (int t1 = tlo[1]; t1 <= thi[1]; ++t1)
                        for (int t2 = tlo[2]; t2 <= thi[2]; ++t2) {
                            if (A == B && (t0 < 0 || (t0 == 0 && (t1 < 0 || (t1 == 0 && t2 < 0))))) continue;
                            const Vec3 sh = G.lat(t0, t1, t2);
                            const Vec3 cb = add(CB.c, sh);
                            const Vec3 d = sub(CA.c, cb);
                            if (dot(d, d) >= reach * reach) continue;
                            // atom pairs and their blocks
                            PairOutT<CL> po;
                            GPairT<CL> &P = po.pair;
                            std::memset(&P, 0, sizeof(P));
                            for (int k = 0; k < CL; ++k) { P.a[k] = -1; P.b[k] = -1; }
                            for (size_t k = 0; k < CA.atoms.size(); ++k) P.a[k] = CA.atoms[k];
                            for (size_t k = 0; k < CB.atoms.size(); ++k) P.b[k] = CB.atoms[k];
                            P.shiftA[0] = P.shiftA[1] = P.shiftA[2] = 0.0;
                            P.shiftB[0] = sh.x; P.shiftB[1] = sh.y; P.shiftB[2] = sh.z;
                            P.self = (A == B && t0 == 0 && t1 == 0 && t2 == 0) ? 1 : 0;
                            bool any_overlap = false;
                            for (int ia = 0; ia < CL; ++ia)
                                for (int jb = 0; jb < CL; ++jb) {
                                    P.hoff[ia * CL + jb] = -1;
                                    P.hoff_t[ia * CL + jb] = -1;
                                    const int a = P.a[ia], b = P.b[jb];
                                    if (a < 0 || b < 0) continue;
                                    const Vec3 dab = sub(pos[a], add(pos[b], sh));
                                    const bool near = dot(dab, dab) < (rc[a] + rc[b]) * (rc[a] + rc[b]);
                                    const long long o = bm.find(a, b, t0, t1, t2);
                                    const long long ot = bm.find(b, a, -t0, -t1, -t2);
                                    P.hoff[ia * CL + jb] = o;
                                    P.hoff_t[ia * CL + jb] = ot;
                                    if (near) {
                                        any_overlap = true;
                                        if (o < 0 || ot < 0) {
                                            // missing block: an error only if some grid point lies in both spheres
                                            const double ra = rc[a], rbb = rc[b];
                                            const Vec3 pb = add(pos[b], sh);
                                            long long lo[3], hi[3];
                                            for (int k = 0; k < 3; ++k) {
                                                const double u = G.frac(pos[a], k), ext = ra / G.spacing[k];
                                                lo[k] = (long long)std::floor((u - ext) * G.N[k]) - 1;
                                                hi[k] = (long long)std::ceil((u + ext) * G.N[k]) + 1;
                                            }
                                            bool hit = false;
                                            for (long long n0 = lo[0]; n0 <= hi[0] && !hit; ++n0)
                                                for (long long n1 = lo[1]; n1 <= hi[1] && !hit; ++n1)
                                                    for (long long n2 = lo[2]; n2 <= hi[2] && !hit; ++n2) {
                                                        const Vec3 r = G.point((double)n0, (double)n1, (double)n2);
                                                        const Vec3 xa = sub(r, pos[a]), xb = sub(r, pb);
                                                        if (std::sqrt(dot(xa, xa)) < ra && std::sqrt(dot(xb, xb)) < rbb) hit = true;
                                                    }
                                            if (hit) {
                                                int expected = GINT_OK;
                                                err.compare_exchange_strong(expected, GINT_EPATTERN);
                                            }
                                        }
                                    }
                                }
                            if (!any_overlap) continue;
                            // bigcells in the intersection of the two clusters' reach
                            long long blo[3], bhi[3];
                            for (int k = 0; k < 3; ++k) {
                                const double ua = G.frac(CA.c, k), ub = G.frac(cb, k);
                                const double ea = (CA.reach + Rb) / G.spacing[k], eb = (CB.reach + Rb) / G.spacing[k];
                                const double lo = std::max(ua - ea, ub - eb), hi = std::min(ua + ea, ub + eb);
                                blo[k] = (long long)std::floor(lo * G.N[k] / GINT_BC) - 1;
                                bhi[k] = (long long)std::ceil(hi * G.N[k] / GINT_BC) + 1;
                            }
                            // along a3 the bigcell centre is c0 + b2 v; an atom's sphere
                            // of radius R holds it for b2 between the roots of
                            // |c0 - p + b2 v|^2 = R^2.  The hull of those intervals over
                            // a cluster, widened by one bigcell, bounds the b2 the exact
                            // test below can accept, so only they are tested
                            const Vec3 v{GINT_BC * G.e[2].x, GINT_BC * G.e[2].y, GINT_BC * G.e[2].z};
                            const double vv = dot(v, v);
                            auto hull = [&](const Cluster &C, const Vec3 &shift, const Vec3 &c0, double &lo, double &hi) {
                                lo = 1e300;
                                hi = -1e300;
                                for (int a : C.atoms) {
                                    const Vec3 d = sub(c0, add(pos[a], shift));
                                    const double R = rc[a] + Rb;
                                    const double bq = dot(d, v), disc = bq * bq - vv * (dot(d, d) - R * R);
                                    if (disc < 0) continue;
                                    const double sq = std::sqrt(disc);
                                    lo = std::min(lo, (-bq - sq) / vv);
                                    hi = std::max(hi, (-bq + sq) / vv);
                                }
                            };
                            const Vec3 zero{0.0, 0.0, 0.0};
                            for (long long b0 = blo[0]; b0 <= bhi[0]; ++b0) {
                                if (!slab.has((int)(((GINT_BC * b0) % G.N[0] + G.N[0]) % G.N[0]), G.N[0])) continue;
                                for (long long b1 = blo[1]; b1 <= bhi[1]; ++b1) {
                                    const Vec3 c0 = G.point(GINT_BC * b0 + 1.5, GINT_BC * b1 + 1.5, 1.5);
                                    double la, ha, lb, hb;
                                    hull(CA, zero, c0, la, ha);
                                    if (la > ha) continue;
                                    hull(CB, sh, c0, lb, hb);
                                    if (lb > hb) continue;
                                    const double zl = std::max(la, lb), zh = std::min(ha, hb);
                                    if (zl > zh + 2.0) continue;
                                    const long long z0 = std::max(blo[2], (long long)std::floor(zl) - 1);
                                    const long long z1 = std::min(bhi[2], (long long)std::ceil(zh) + 1);
                                    for (long long b2 = z0; b2 <= z1; ++b2) {
                                        const Vec3 ctr = G.point(GINT_BC * b0 + 1.5, GINT_BC * b1 + 1.5, GINT_BC * b2 + 1.5);
                                        bool ina = false, inb = false;
                                        for (int a : CA.atoms) {
                                            const Vec3 x = sub(ctr, pos[a]);
                                            const double R = rc[a] + Rb;
                                            if (dot(x, x) < R * R) { ina = true; break; }
                                        }
                                        if (!ina) continue;
                                        for (int b : CB.atoms) {
                                            const Vec3 x = sub(ctr, add(pos[b], sh));
                                            const double R = rc[b] + Rb;
                                            if (dot(x, x) < R * R) { inb = true; break; }
                                        }
                                        if (!inb) continue;
                                        if (std::llabs(b0) > (1LL << 28) || std::llabs(b1) > (1LL << 28) || std::llabs(b2) > (1LL << 28)) {
                                            int expected = GINT_OK;
                                            err.compare_exchange_strong(expected, GINT_EINVAL);
                                            continue;
                                        }
                                        po.bcs.push_back(make_bigcell(G.N, GINT_BC * b0, GINT_BC * b1, GINT_BC * b2));
                                    }
                                }
                            }
                            if (!po.bcs.empty()) per_a[A].push_back(std::move(po));
                        }
            }
        }
    };
    unsigned nth = std::thread::hardware_concurrency();
    if (nth == 0) nth = 4;
    nth = std::min(nth, 16u);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t) th.emplace_back(worker);
    for (auto &t : th) t.join();
    if (err.load() != GINT_OK)
        return fail(err.load(), err.load() == GINT_EPATTERN ? "an overlapping (I,J,R) block is missing from the pattern"
                                                            : "grid index out of range");

    // ---- flatten: canonical pairs, then their swapped copies.  Offsets per
    // A cluster first, then each A's pairs and bigcell lists are copied by a
    // worker into place.
    pairs.clear();
    hp.bigcells.clear();
    std::vector<size_t> pair_at(ncl + 1, 0), bc_at(ncl + 1, 0);
    for (int A = 0; A < ncl; ++A) {
        size_t nb = 0;
        for (auto &po : per_a[A]) nb += po.bcs.size();
        pair_at[A + 1] = pair_at[A] + per_a[A].size();
        bc_at[A + 1] = bc_at[A] + nb;
    }
    const size_t npair = pair_at[ncl], nbc = bc_at[ncl];
    if (nbc > (size_t)0x7fffffff) return fail(GINT_ENOMEM, "too many bigcells");
    pairs.reserve(with_swapped ? 2 * npair : npair);
    pairs.resize(npair);
    hp.bigcells.resize(nbc);
    std::vector<std::pair<int, int>> ranges(npair);   // per canonical pair: bigcell begin, count
    parallel_for(ncl, [&](int A) {
        size_t p = pair_at[A], b = bc_at[A];
        for (auto &po : per_a[A]) {
            ranges[p] = {(int)b, (int)po.bcs.size()};
            std::copy(po.bcs.begin(), po.bcs.end(), hp.bigcells.begin() + b);
            pairs[p] = po.pair;
            ++p;
            b += po.bcs.size();
        }
        std::vector<PairOutT<CL>>().swap(per_a[A]);
    });
    hp.ncanon = (int)pairs.size();
    std::vector<int> swapped_of(hp.ncanon, -1);
    for (int p = 0; p < hp.ncanon && with_swapped; ++p) {
        const GPairT<CL> P = pairs[p];
        if (P.self) continue;
        GPairT<CL> S;
        std::memset(&S, 0, sizeof(S));
        for (int k = 0; k < CL; ++k) { S.a[k] = P.b[k]; S.b[k] = P.a[k]; }
        for (int k = 0; k < 3; ++k) { S.shiftA[k] = P.shiftB[k]; S.shiftB[k] = P.shiftA[k]; }
        S.self = 0;
        for (int i = 0; i < CL; ++i)
            for (int j = 0; j < CL; ++j) {
                S.hoff[i * CL + j] = P.hoff_t[j * CL + i];
                S.hoff_t[i * CL + j] = P.hoff[j * CL + i];
            }
        swapped_of[p] = (int)pairs.size();
        pairs.push_back(S);
    }

    // ---- work items: runs of at most maxbc bigcells, longest first.  With
    // enough pairs to fill the GPU several times over, a pair is one item
    // (exclusive: its H blocks are written with plain stores); otherwise long
    // pairs are split for load balance.
    long long total_bc = 0;
    int longest = 0;
    for (int p = 0; p < hp.ncanon; ++p) {
        total_bc += ranges[p].second;
        longest = std::max(longest, ranges[p].second);
    }
    int maxbc = maxbc_opt;
    if (maxbc <= 0) {
        const long long slots = 2048;    // resident workgroups of a large GPU, with margin
        const long long per_slot = (total_bc + slots - 1) / slots;
        maxbc = (int)std::max<long long>(64, std::min<long long>(std::max<long long>(per_slot, 64), 1LL << 30));
        if (longest <= per_slot * 2) maxbc = std::max(maxbc, longest);
    }
    hp.items_canon.clear();
    hp.items_ordered.clear();
    for (int p = 0; p < hp.ncanon; ++p) {
        const int beg = ranges[p].first, cnt = ranges[p].second;
        const int nchunk = (cnt + maxbc - 1) / maxbc;
        const int excl = (nchunk == 1 && slab.count <= 1) ? 1 : 0;
        for (int c = 0; c < nchunk; ++c) {
            const int b0 = beg + (int)((long long)cnt * c / nchunk);
            const int b1 = beg + (int)((long long)cnt * (c + 1) / nchunk);
            hp.items_canon.push_back({p, b0, b1 - b0, excl});
            hp.items_ordered.push_back({p, b0, b1 - b0, excl});
            if (swapped_of[p] >= 0) hp.items_ordered.push_back({swapped_of[p], b0, b1 - b0, excl});
        }
    }
    auto longer = [](const GItem &x, const GItem &y) {
        if (x.bc_count != y.bc_count) return x.bc_count > y.bc_count;
        if (x.pair != y.pair) return x.pair < y.pair;
        return x.bc_begin < y.bc_begin;
    };
    std::sort(hp.items_canon.begin(), hp.items_canon.end(), longer);
    std::sort(hp.items_ordered.begin(), hp.items_ordered.end(), longer);

    return GINT_OK;
}

static int build_one(const gint_system *sys, const gint_options *opt, bool bricks, const GintSlab &slab,
                     HostPlan &hp) {
    auto fail = [&](int code, const char *msg) {
        hp.error = msg;
        return code;
    };
    if (!sys) return fail(GINT_EINVAL, "null system");
    // clusters of up to eight atoms serve only the eight-wave mixed Vlocal,
    // i.e. plans whose rho and force run on bricks.  The default is four: on
    // the bilayers a pair of eight-atom clusters covers half as many bigcells
    // as four pairs of four-atom ones, so the orbital evaluations, which
    // bound Vlocal, do not drop, and the per-bigcell overhead doubles.
    const bool wide_ok = opt && opt->precision != GINT_FP64 &&
                         (opt->decomposition == GINT_DECOMP_DEFAULT || opt->decomposition == GINT_DECOMP_BIGCELL_RHO_FORCE);
    const int cl = (opt && opt->cluster_atoms > 0) ? opt->cluster_atoms : GINT_CL;
    if (cl < 1 || cl > GINT_CL8) return fail(GINT_EINVAL, "cluster_atoms out of range");
    if (cl > GINT_CL && !wide_ok)
        return fail(GINT_EINVAL, "clusters of more than 4 atoms need a mixed-precision plan with bigcell rho/force");
    const int maxbc_opt = (opt && opt->max_bigcells_per_item > 0) ? opt->max_bigcells_per_item : 0;
    hp.cluster_atoms = cl;
    if (sys->natom < 1 || !sys->pos || !sys->species) return fail(GINT_EINVAL, "bad atoms");
    if (sys->nspecies < 1 || sys->nspecies > GINT_MAXSPECIES || !sys->species_list)
        return fail(GINT_EINVAL, "bad species list");
    for (int k = 0; k < 3; ++k)
        if (sys->grid[k] < 1) return fail(GINT_EINVAL, "grid must be positive");
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(sys->cell[k])) return fail(GINT_EINVAL, "non-finite cell");

    Geometry G;
    std::memcpy(G.cell, sys->cell, sizeof(G.cell));
    double det;
    if (!invert3(G.cell, G.inv, &det)) return fail(GINT_EINVAL, "singular cell");
    for (int i = 0; i < 3; ++i) {
        G.N[i] = sys->grid[i];
        G.a[i] = {G.cell[3 * i], G.cell[3 * i + 1], G.cell[3 * i + 2]};
        G.e[i] = {G.a[i].x / G.N[i], G.a[i].y / G.N[i], G.a[i].z / G.N[i]};
        const double bx = G.inv[i], by = G.inv[3 + i], bz = G.inv[6 + i];
        G.spacing[i] = 1.0 / std::sqrt(bx * bx + by * by + bz * bz);
    }
    hp.omega = std::fabs(det);
    hp.ngrid = (long long)G.N[0] * G.N[1] * G.N[2];
    hp.w = hp.omega / (double)hp.ngrid;
    std::memcpy(hp.cell, G.cell, sizeof(hp.cell));
    for (int i = 0; i < 3; ++i) {
        hp.N[i] = G.N[i];
        hp.e[i][0] = G.e[i].x; hp.e[i][1] = G.e[i].y; hp.e[i][2] = G.e[i].z;
    }

    // ---- species and radial tables ([knot][chan][f, f'] interleaved)
    hp.species.clear();
    hp.tab.clear();
    for (int s = 0; s < sys->nspecies; ++s) {
        const gint_species &sp = sys->species_list[s];
        if (!(sp.rcut > 0) || !(sp.dr > 0) || sp.nknots < 2 || sp.nchan < 1 || sp.nchan > GINT_MAXCHAN ||
            !sp.chan_l || !sp.f || !sp.fp || !std::isfinite(sp.rcut) || !std::isfinite(sp.dr))
            return fail(GINT_EINVAL, "bad species");
        if ((sp.nknots - 1) * sp.dr < sp.rcut * (1.0 - 1e-12)) return fail(GINT_EINVAL, "table shorter than rcut");
        GSpecies g{};
        g.rcut = sp.rcut;
        g.rcut2 = sp.rcut * sp.rcut;
        g.dr = sp.dr;
        g.inv_dr = 1.0 / sp.dr;
        g.nknots = sp.nknots;
        g.nchan = sp.nchan;
        int norb = 0;
        for (int c = 0; c < sp.nchan; ++c) {
            if (sp.chan_l[c] < 0) return fail(GINT_EINVAL, "negative l");
            if (sp.chan_l[c] > 2) return fail(GINT_EUNSUPPORTED, "l > 2 not supported");
            g.chan_l[c] = sp.chan_l[c];
            norb += 2 * sp.chan_l[c] + 1;
        }
        if (norb > GINT_ORB) return fail(GINT_EUNSUPPORTED, "more than 16 orbitals per atom");
        g.norb = norb;
        {
            const int *l = sp.chan_l;
            if (sp.nchan == 5 && l[0] == 0 && l[1] == 0 && l[2] == 1 && l[3] == 1 && l[4] == 2)
                g.shape = GINT_SHAPE_2S2P1D;
            else if (sp.nchan == 3 && l[0] == 0 && l[1] == 0 && l[2] == 1)
                g.shape = GINT_SHAPE_2S1P;
            else
                g.shape = GINT_SHAPE_ANY;
        }
        g.tab_off = (int)hp.tab.size();
        // bound on |phi| = |p_c(r)| |S_lm(x)| over the table: the Hermite
        // cubic on [r_k, r_k+1] is at most |f_k| + |f_k+1| + (4/27) dr
        // (|f'_k| + |f'_k+1|), and |S_lm(x)| <= r^l sqrt((2l+1)/(4 pi))
        for (int c = 0; c < sp.nchan; ++c) {
            const int l = sp.chan_l[c];
            const double ylm = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
            const double *f = sp.f + (size_t)c * sp.nknots, *fp = sp.fp + (size_t)c * sp.nknots;
            for (int k = 0; k + 1 < sp.nknots && k * sp.dr < sp.rcut; ++k) {
                const double pk = std::fabs(f[k]) + std::fabs(f[k + 1]) +
                                  (4.0 / 27.0) * sp.dr * (std::fabs(fp[k]) + std::fabs(fp[k + 1]));
                const double r1 = std::min((k + 1) * sp.dr, sp.rcut);
                const double b = pk * std::pow(r1, l) * ylm;
                if (std::isfinite(b) && b > hp.phi_max) hp.phi_max = b;
            }
        }
        for (int k = 0; k < sp.nknots; ++k)
            for (int c = 0; c < sp.nchan; ++c) {
                const double f = sp.f[(size_t)c * sp.nknots + k], fp = sp.fp[(size_t)c * sp.nknots + k];
                if (!std::isfinite(f) || !std::isfinite(fp)) return fail(GINT_EINVAL, "non-finite radial table");
                hp.tab.push_back(f);
                hp.tab.push_back(fp);
            }
        hp.species.push_back(g);
    }
    if (hp.tab.size() > (size_t)0x7fffffff) return fail(GINT_EINVAL, "radial tables too large");
    // FP32 tables by knot interval: [interval k][chan][c0, c1, c2, c3], the
    // coefficients of the same cubic Hermite interpolant as a polynomial in
    // t = r/dr - k, p = c0 + c1 t + c2 t^2 + c3 t^3, times the normalisation
    // constant of the channel's solid harmonics (K_0 = 1/(2 sqrt(pi)),
    // K_1 = sqrt(3/(4 pi)), K_2 = sqrt(15/pi)/2), computed in FP64 and
    // rounded once.  Folding K_l in here keeps it out of the FP32 arithmetic:
    // rounded to FP32 on its own, K_0 and K_2 carry a relative error of
    // 5e-8 that every orbital of the channel would share, a bias that does
    // not average out over grid points (it doubled on diagonal H elements,
    // where both operands carry it).  In this form p' = (c1 + 2 c2 t + 3 c3 t^2)/dr has no
    // cancellation: the weighted-knot form h00' f_k + h01' f_k+1 cancels two
    // terms of size 6 f/dr, which in FP32 cost about 8 bits of the gradient.
    // 16-byte records, so one evaluation reads each channel with one 16-byte
    // load.  Twice the length of the FP64 table, so species s starts at
    // 2 tab_off (also after the batch merge); the record of the last knot
    // (never an interval start) holds the constant f_k.
    hp.tab32.assign(2 * hp.tab.size(), 0.f);
    for (const GSpecies &g : hp.species) {
        const size_t C = (size_t)g.nchan, K = (size_t)g.nknots;
        const double *t = hp.tab.data() + g.tab_off;
        float *o = hp.tab32.data() + 2 * (size_t)g.tab_off;
        for (size_t k = 0; k < K; ++k) {
            for (size_t c = 0; c < C; ++c) {
                const int l = g.chan_l[c];
                const double kl = l == 0 ? 0.5 / std::sqrt(M_PI)
                                         : (l == 1 ? std::sqrt(3.0 / (4.0 * M_PI)) : 0.5 * std::sqrt(15.0 / M_PI));
                float *r = o + (k * C + c) * 4;
                const double f0 = t[(k * C + c) * 2], d0 = g.dr * t[(k * C + c) * 2 + 1];
                if (k + 1 < K) {
                    const double f1 = t[((k + 1) * C + c) * 2], d1 = g.dr * t[((k + 1) * C + c) * 2 + 1];
                    r[0] = (float)(kl * f0);
                    r[1] = (float)(kl * d0);
                    r[2] = (float)(kl * (3.0 * (f1 - f0) - 2.0 * d0 - d1));
                    r[3] = (float)(kl * (2.0 * (f0 - f1) + d0 + d1));
                } else {
                    r[0] = (float)(kl * f0);
                    r[1] = r[2] = r[3] = 0.f;
                }
            }
        }
    }

    // ---- atoms
    const int natom = sys->natom;
    hp.natom = natom;
    std::vector<Vec3> pos(natom);
    std::vector<double> rc(natom);
    std::vector<int> norb(natom);
    hp.atoms.resize(natom);
    double rcmax = 0;
    for (int i = 0; i < natom; ++i) {
        const int s = sys->species[i];
        if (s < 0 || s >= sys->nspecies) return fail(GINT_EINVAL, "species index out of range");
        pos[i] = {sys->pos[3 * i], sys->pos[3 * i + 1], sys->pos[3 * i + 2]};
        if (!std::isfinite(pos[i].x) || !std::isfinite(pos[i].y) || !std::isfinite(pos[i].z))
            return fail(GINT_EINVAL, "non-finite position");
        rc[i] = hp.species[s].rcut;
        norb[i] = hp.species[s].norb;
        rcmax = std::max(rcmax, rc[i]);
        hp.atoms[i] = {pos[i].x, pos[i].y, pos[i].z, s, norb[i]};
    }
    if (natom >= (1 << 22)) return fail(GINT_EINVAL, "too many atoms");

    // ---- pattern (validated and indexed once per system when slabs share it)
    if (sys->nblk < 0 || (sys->nblk > 0 && (!sys->blk_i || !sys->blk_j || !sys->blk_r || !sys->blk_off)))
        return fail(GINT_EINVAL, "bad pattern arrays");
    BlockMap bm_local;
    const BlockMap *bmp = &bm_local;
    if (slab.shared && slab.shared->pattern) {
        bmp = &slab.shared->bm;
        hp.nnz = slab.shared->nnz;
    } else {
        BlockMap &bm = bm_local;
        bm.reserve((size_t)sys->nblk);
        std::vector<std::pair<long long, long long>> spans;
        spans.reserve(sys->nblk);
        long long nnz = 0;
        for (int b = 0; b < sys->nblk; ++b) {
            const int i = sys->blk_i[b], j = sys->blk_j[b];
            const int *r = sys->blk_r + 3 * b;
            if (i < 0 || i >= natom || j < 0 || j >= natom) return fail(GINT_EINVAL, "block atom out of range");
            if (std::abs(r[0]) >= 2048 || std::abs(r[1]) >= 2048 || std::abs(r[2]) >= 2048)
                return fail(GINT_EINVAL, "block R out of range");
            const long long off = sys->blk_off[b];
            const long long sz = (long long)norb[i] * norb[j];
            if (off < 0) return fail(GINT_EINVAL, "negative block offset");
            if (!bm.insert(BlockKey{i, j, r[0], r[1], r[2]}, off)) return fail(GINT_EINVAL, "duplicate block");
            spans.push_back({off, off + sz});
            nnz = std::max(nnz, off + sz);
        }
        std::sort(spans.begin(), spans.end());
        for (size_t k = 1; k < spans.size(); ++k)
            if (spans[k].first < spans[k - 1].second) return fail(GINT_EINVAL, "overlapping blocks");
        hp.blocks.resize(sys->nblk);
        for (int b = 0; b < sys->nblk; ++b) {
            const int *r = sys->blk_r + 3 * b;
            const long long ot = bm.find(sys->blk_j[b], sys->blk_i[b], -r[0], -r[1], -r[2]);
            if (ot < 0) return fail(GINT_EPATTERN, "pattern is not transpose-closed");
            hp.blocks[b] = GBlk{sys->blk_off[b], ot, norb[sys->blk_i[b]], norb[sys->blk_j[b]], 0, sys->blk_i[b],
                                sys->blk_j[b], 0};
        }
        hp.nnz = nnz;
        if (slab.shared) {
            slab.shared->bm = std::move(bm_local);
            slab.shared->nnz = nnz;
            slab.shared->pattern = true;
            bmp = &slab.shared->bm;
        }
    }
    const BlockMap &bm = *bmp;

    // ---- clusters, cluster pairs and their work items
    const double Rb = bigcell_radius(G);
    {
        const int r = cl > GINT_CL
                          ? build_cluster_pairs<GINT_CL8>(G, pos, rc, bm, cl, maxbc_opt, Rb, false, slab, hp.pairs8, hp)
                          : build_cluster_pairs<GINT_CL>(G, pos, rc, bm, cl, maxbc_opt, Rb, true, slab, hp.pairs, hp);
        if (r != GINT_OK) return r;
    }

    // ---- bigcell-stationary bricks.  Default shape: about 2 Bohr along each
    // axis (anisotropic grids get anisotropic bricks), at most 8 bigcells;
    // halved along the longest axis while a union exceeds GINT_UMAX.
    if (bricks) {
        int B[3];
        for (int k = 0; k < 3; ++k) {
            const int req = opt ? opt->brick[k] : 0;
            if (req < 0 || req > 8) return fail(GINT_EINVAL, "brick dimension out of range (1..8)");
            if (req > 0) {
                B[k] = req;
            } else {
                const double hk = std::sqrt(dot(G.e[k], G.e[k]));
                B[k] = (int)std::lround(2.0 / (4.0 * hk));
                B[k] = std::max(1, std::min(8, B[k]));
            }
        }
        BlockIndex bidx_local;
        const BlockIndex *bidxp = &bidx_local;
        if (slab.shared && slab.shared->index) {
            bidxp = &slab.shared->bidx;
        } else {
            bidx_local.build(sys->nblk, sys->blk_i, sys->blk_j, sys->blk_r);
            if (slab.shared) {
                slab.shared->bidx = std::move(bidx_local);
                slab.shared->index = true;
                bidxp = &slab.shared->bidx;
            }
        }
        const BlockIndex &bidx = *bidxp;
        std::vector<int> spec(natom);
        for (int i = 0; i < natom; ++i) spec[i] = sys->species[i];
        for (;;) {
            const int r = build_bricks(G, pos, rc, spec, bidx, B, Rb, slab, hp);
            if (r == GINT_OK) break;
            if (r != 1) return fail(r, "grid too large for the brick index");
            int ax = 0;
            for (int k = 1; k < 3; ++k)
                if (B[k] > B[ax]) ax = k;
            if (B[ax] == 1)
                return fail(GINT_EUNSUPPORTED, "more atom images reach one bigcell than the kernels hold (256)");
            B[ax] = (B[ax] + 1) / 2;
        }
        for (int k = 0; k < 3; ++k) hp.brick[k] = B[k];
    }
    return GINT_OK;
}

// Appends the cluster pairs of system i of a batch, with its atom and
// matrix offsets applied.
template <int CL>
void merge_pairs(const std::vector<GPairT<CL>> &src, int i, int atom_off, long long nnz_off,
                 std::vector<GPairT<CL>> &dst) {
    for (GPairT<CL> P : src) {
        for (int k = 0; k < CL; ++k) {
            if (P.a[k] >= 0) P.a[k] += atom_off;
            if (P.b[k] >= 0) P.b[k] += atom_off;
        }
        for (int k = 0; k < CL * CL; ++k) {
            if (P.hoff[k] >= 0) P.hoff[k] += nnz_off;
            if (P.hoff_t[k] >= 0) P.hoff_t[k] += nnz_off;
        }
        P.sys = i;
        dst.push_back(P);
    }
}

int gint_build_host_plan(const gint_system *sys, int n_sys, const gint_options *opt, bool bricks, HostPlan &hp,
                         const GintSlab *slab_in) {
    if (!sys || n_sys < 1) {
        hp.error = "no systems";
        return GINT_EINVAL;
    }
    const GintSlab slab = slab_in ? *slab_in : GintSlab{};
    if (slab.count < 1 || slab.index < 0 || slab.index >= slab.count || (slab.count > 1 && n_sys != 1)) {
        hp.error = "bad slab";
        return GINT_EINVAL;
    }
    hp = HostPlan();
    // every system's plan first, then each merged array is reserved once at
    // its final size (growing them system by system re-copied them)
    std::vector<HostPlan> ones((size_t)n_sys);
    for (int i = 0; i < n_sys; ++i) {
        const int rc = build_one(sys + i, opt, bricks, slab, ones[(size_t)i]);
        if (rc != GINT_OK) {
            hp.error = "system " + std::to_string(i) + ": " + ones[(size_t)i].error;
            return rc;
        }
    }
    if (n_sys > 1) {
        size_t nb = 0, nsp = 0, nt = 0, nt32 = 0, na = 0, np = 0, np8 = 0, nbc = 0, nbk = 0, nu = 0, npt = 0, nic = 0,
               nio = 0;
        for (const HostPlan &o : ones) {
            nb += o.blocks.size(); nsp += o.species.size(); nt += o.tab.size(); nt32 += o.tab32.size();
            na += o.atoms.size(); np += o.pairs.size(); np8 += o.pairs8.size(); nbc += o.bigcells.size();
            nbk += o.bricks.size(); nu += o.uatoms.size(); npt += o.ptab.size(); nic += o.items_canon.size();
            nio += o.items_ordered.size();
        }
        hp.blocks.reserve(nb); hp.species.reserve(nsp); hp.tab.reserve(nt); hp.tab32.reserve(nt32);
        hp.atoms.reserve(na); hp.pairs.reserve(np); hp.pairs8.reserve(np8); hp.bigcells.reserve(nbc);
        hp.bricks.reserve(nbk); hp.uatoms.reserve(nu); hp.ptab.reserve(npt); hp.items_canon.reserve(nic);
        hp.items_ordered.reserve(nio); hp.sys.reserve((size_t)n_sys);
    }
    long long g_off = 0, nnz_off = 0;
    int atom_off = 0, species_off = 0;
    long long tab_off = 0;
    for (int i = 0; i < n_sys; ++i) {
        HostPlan one = std::move(ones[(size_t)i]);
        GSys S{};
        for (int k = 0; k < 3; ++k) {
            S.N[k] = one.N[k];
            for (int m = 0; m < 3; ++m) S.e[k][m] = one.e[k][m];
        }
        S.natom = one.natom;
        S.w = one.w;
        S.volume = one.omega;
        S.g_off = g_off;
        S.nnz_off = nnz_off;
        S.atom_off = atom_off;
        if (i == 0) {
            for (int k = 0; k < 3; ++k) hp.N[k] = one.N[k];
            std::memcpy(hp.e, one.e, sizeof(hp.e));
            std::memcpy(hp.cell, one.cell, sizeof(hp.cell));
            hp.w = one.w;
            hp.omega = one.omega;
            hp.cluster_atoms = one.cluster_atoms;
        }
        hp.sys.push_back(S);
        hp.phi_max = std::max(hp.phi_max, one.phi_max);
        const size_t n_species = one.species.size(), n_tab = one.tab.size();
        if (i > 0 && one.pairs8.empty() != hp.pairs8.empty()) {
            hp.error = "systems of one plan must share the cluster size";
            return GINT_EINVAL;
        }
        if (n_sys == 1) {
            // a single system's offsets are all zero: its arrays are taken
            // as they are (no copy of the bigcell lists and pair tables)
            hp.blocks = std::move(one.blocks);
            hp.species = std::move(one.species);
            hp.tab = std::move(one.tab);
            hp.tab32 = std::move(one.tab32);
            hp.atoms = std::move(one.atoms);
            hp.pairs = std::move(one.pairs);
            hp.pairs8 = std::move(one.pairs8);
            hp.bigcells = std::move(one.bigcells);
            hp.bricks = std::move(one.bricks);
            hp.uatoms = std::move(one.uatoms);
            hp.ptab = std::move(one.ptab);
            hp.items_canon = std::move(one.items_canon);
            hp.items_ordered = std::move(one.items_ordered);
            for (int k = 0; k < 3; ++k) hp.brick[k] = one.brick[k];
        } else {
            for (GBlk b : one.blocks) {
                b.off += nnz_off;
                b.off_t += nnz_off;
                b.sys = i;
                b.i += atom_off;
                b.j += atom_off;
                hp.blocks.push_back(b);
            }
            for (GSpecies sp : one.species) {
                sp.tab_off += (int)tab_off;
                hp.species.push_back(sp);
            }
            hp.tab.insert(hp.tab.end(), one.tab.begin(), one.tab.end());
            hp.tab32.insert(hp.tab32.end(), one.tab32.begin(), one.tab32.end());
            for (GAtom at : one.atoms) {
                at.species += species_off;
                hp.atoms.push_back(at);
            }
            const int pair_off = (int)(hp.pairs.size() + hp.pairs8.size());
            const int bc_off = (int)hp.bigcells.size();
            if (hp.bigcells.size() + one.bigcells.size() > (size_t)0x7fffffff) {
                hp.error = "too many bigcells";
                return GINT_ENOMEM;
            }
            merge_pairs(one.pairs, i, atom_off, nnz_off, hp.pairs);
            merge_pairs(one.pairs8, i, atom_off, nnz_off, hp.pairs8);
            hp.bigcells.insert(hp.bigcells.end(), one.bigcells.begin(), one.bigcells.end());
            {
                const int ub = (int)hp.uatoms.size();
                const long long pb = (long long)hp.ptab.size();
                const int blk_base = (int)(hp.blocks.size() - one.blocks.size());
                if (hp.uatoms.size() + one.uatoms.size() > (size_t)0x7fffffff) {
                    hp.error = "too many atom images in the bricks";
                    return GINT_ENOMEM;
                }
                for (GBrick b : one.bricks) {
                    b.sys = i;
                    b.u_begin += ub;
                    b.pt_off += pb;
                    hp.bricks.push_back(b);
                }
                for (GUAtom u : one.uatoms) {
                    u.atom += atom_off;
                    u.species += species_off;
                    hp.uatoms.push_back(u);
                }
                const size_t pt0 = hp.ptab.size();
                hp.ptab.resize(pt0 + one.ptab.size());
                for (size_t q = 0; q < one.ptab.size(); ++q) {
                    const int b = one.ptab[q];
                    hp.ptab[pt0 + q] = b >= 0 ? b + blk_base : -1;
                }
            }
            for (GItem it : one.items_canon) {
                it.pair += pair_off;
                it.bc_begin += bc_off;
                hp.items_canon.push_back(it);
            }
            for (GItem it : one.items_ordered) {
                it.pair += pair_off;
                it.bc_begin += bc_off;
                hp.items_ordered.push_back(it);
            }
        }
        hp.ncanon += one.ncanon;
        hp.ncluster += one.ncluster;
        hp.natom += one.natom;
        hp.ngrid += one.ngrid;
        hp.nnz += one.nnz;
        g_off += one.ngrid;
        nnz_off += one.nnz;
        atom_off += one.natom;
        species_off += (int)n_species;
        tab_off += (long long)n_tab;
        if (tab_off > 0x7fffffffLL) {
            hp.error = "radial tables too large";
            return GINT_EINVAL;
        }
    }
    if (n_sys > 1) {
        auto longer = [](const GItem &x, const GItem &y) {
            if (x.bc_count != y.bc_count) return x.bc_count > y.bc_count;
            if (x.pair != y.pair) return x.pair < y.pair;
            return x.bc_begin < y.bc_begin;
        };
        std::sort(hp.items_canon.begin(), hp.items_canon.end(), longer);
        std::sort(hp.items_ordered.begin(), hp.items_ordered.end(), longer);
    }
    return GINT_OK;
}
