// Host construction of the IFGF hierarchy (Sec. 3.3.1-3.3.2): root box,
// Morton-ordered points, relevant boxes of every level as contiguous Morton
// ranges, parents/children, neighbours and cousins, cone intervals per
// level, and the relevant cone segments of every box with their slot tables.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <thread>

#include <sys/mman.h>

#include "host_mem.hpp"
#include "ifgf_internal.hpp"

namespace ifgf {
namespace {

// IFGF_PLAN_TIMES=1: seconds of each phase of the construction on stderr
// (per building thread).
struct PhaseClock {
    bool on = false;
    std::chrono::steady_clock::time_point t;
    void start()
    {
        const char* e = std::getenv("IFGF_PLAN_TIMES");
        on = e && std::atoi(e) != 0;
        t = std::chrono::steady_clock::now();
    }
    void lap(const char* what)
    {
        auto n = std::chrono::steady_clock::now();
        if (on) std::fprintf(stderr, "plan: %-36s %8.3f s\n", what, std::chrono::duration<double>(n - t).count());
        t = n;
    }
};
thread_local PhaseClock g_clock;

int host_threads()
{
    const char* e = std::getenv("IFGF_HOST_THREADS");
    int t = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
    if (t < 1) t = 1;
    if (t > 16) t = 16;
    return t;
}

// Runs f(i) for i in [0, n) on a small thread pool, `grain` indices at a time.
template <class F>
void parallel_for(int64_t n, F&& f, int64_t grain = 1)
{
    int nt = host_threads();
    if (n <= grain || nt == 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (;;) {
            int64_t b = next.fetch_add(grain);
            if (b >= n) break;
            int64_t e = std::min(n, b + grain);
            for (int64_t i = b; i < e; ++i) f(i);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
}

}  // namespace

void map_pages(void* p, size_t bytes)
{
    if (bytes < ((size_t)16 << 20)) return;
    const uintptr_t pg = 4096, huge = (uintptr_t)2 << 20, chunk = (uintptr_t)32 << 20;
    const uintptr_t a = ((uintptr_t)p + pg - 1) & ~(pg - 1);
    const uintptr_t b = ((uintptr_t)p + bytes) & ~(pg - 1);
    if (b <= a) return;
    madvise((void*)a, b - a, MADV_HUGEPAGE);
    // chunks aligned to the huge page, one thread each
    const uintptr_t a0 = a & ~(huge - 1);
    const int64_t nchunk = (int64_t)((b - a0 + chunk - 1) / chunk);
    parallel_for(nchunk, [&](int64_t c) {
        const uintptr_t s = std::max(a, a0 + (uintptr_t)c * chunk);
        const uintptr_t e = std::min(b, a0 + (uintptr_t)(c + 1) * chunk);
        if (s < e) madvise((void*)s, e - s, MADV_POPULATE_WRITE);
    });
}

namespace {

// Stable sort by `less`: chunks sorted on the thread pool, then merged
// pairwise in rounds (each round's merges in parallel; merging keeps the
// order of equal elements).
template <class T, class Less>
void parallel_stable_sort(std::vector<T>& v, Less less)
{
    const int64_t n = (int64_t)v.size();
    int nc = 1;
    while (nc < host_threads()) nc *= 2;
    if (n < (int64_t)1 << 15 || nc == 1) {
        std::stable_sort(v.begin(), v.end(), less);
        return;
    }
    std::vector<int64_t> cut(nc + 1);
    for (int c = 0; c <= nc; ++c) cut[c] = n * c / nc;
    parallel_for(nc, [&](int64_t c) { std::stable_sort(v.begin() + cut[c], v.begin() + cut[c + 1], less); });
    for (int w = 1; w < nc; w *= 2)
        parallel_for(nc / (2 * w), [&](int64_t i) {
            const int64_t a = cut[2 * w * i], m = cut[2 * w * i + w], b = cut[2 * w * (i + 1)];
            std::inplace_merge(v.begin() + a, v.begin() + m, v.begin() + b, less);
        });
}

// Sorts v ascending: chunks sorted on the thread pool, then merged pairwise
// in rounds (each round's merges in parallel).
void parallel_sort(std::vector<uint64_t>& v)
{
    const int64_t n = (int64_t)v.size();
    int nc = 1;
    while (nc < host_threads()) nc *= 2;
    if (n < (int64_t)1 << 16 || nc == 1) {
        std::sort(v.begin(), v.end());
        return;
    }
    std::vector<int64_t> cut(nc + 1);
    for (int c = 0; c <= nc; ++c) cut[c] = n * c / nc;
    parallel_for(nc, [&](int64_t c) { std::sort(v.begin() + cut[c], v.begin() + cut[c + 1]); });
    for (int w = 1; w < nc; w *= 2)
        parallel_for(nc / (2 * w), [&](int64_t i) {
            const int64_t a = cut[2 * w * i], m = cut[2 * w * i + w], b = cut[2 * w * (i + 1)];
            std::inplace_merge(v.begin() + a, v.begin() + m, v.begin() + b);
        });
}

uint64_t interleave3(uint64_t x, uint64_t y, uint64_t z, int bits)
{
    uint64_t c = 0;
    for (int b = 0; b < bits; ++b) {
        c |= ((x >> b) & 1ull) << (3 * b + 2);
        c |= ((y >> b) & 1ull) << (3 * b + 1);
        c |= ((z >> b) & 1ull) << (3 * b);
    }
    return c;
}

void deinterleave3(uint64_t c, int bits, int64_t* k)
{
    k[0] = k[1] = k[2] = 0;
    for (int b = 0; b < bits; ++b) {
        k[0] |= (int64_t)((c >> (3 * b + 2)) & 1ull) << b;
        k[1] |= (int64_t)((c >> (3 * b + 1)) & 1ull) << b;
        k[2] |= (int64_t)((c >> (3 * b)) & 1ull) << b;
    }
}

// Integer part of (x - corner) / H per axis, clamped into [0, nb - 1].
void box_index(const double* x, const double* corner, double H, int64_t nb, int64_t* k)
{
    for (int a = 0; a < 3; ++a) {
        double q = std::floor((x[a] - corner[a]) / H);
        int64_t v = q < 0.0 ? 0 : (int64_t)q;
        k[a] = v > nb - 1 ? nb - 1 : v;
    }
}

int64_t find_prefix(const std::vector<uint64_t>& v, uint64_t key)
{
    auto it = std::lower_bound(v.begin(), v.end(), key);
    if (it == v.end() || *it != key) return -1;
    return (int64_t)(it - v.begin());
}



// Slot of cone (cell, is) of box b, or -1 (host twin of the device lookup).
int32_t host_lookup(const HostLevel& L, int64_t b, int cell, int is)
{
    size_t c = (size_t)b * L.ncell + cell;
    const uint64_t* M = &L.cell_mask[c * L.W];
    int w = is >> 6, bit = is & 63;
    if (!((M[w] >> bit) & 1ull)) return -1;
    int cnt = __builtin_popcountll(M[w] & ((1ull << bit) - 1ull));
    for (int i = 0; i < w; ++i) cnt += __builtin_popcountll(M[i]);
    return L.cell_base[c] + cnt;
}

// First pair of every target box: entry pair_base[T] + c n_T + t is
// (cousin c, target t) of box T.
void pair_offsets(HostLevel& L)
{
    L.pair_base.assign(L.nbox + 1, 0);
    for (int64_t T = 0; T < L.nbox; ++T) {
        int64_t nT = L.box_start[T + 1] - L.box_start[T];
        int64_t cT = L.cou_start[T + 1] - L.cou_start[T];
        L.pair_base[T + 1] = L.pair_base[T] + nT * cT;
    }
}

// Cousin-target pair table of level d (see HostLevel::use_pairs).
void build_pairs(HostPlan& hp, int d)
{
    HostLevel& L = hp.L[d];
    pair_offsets(L);
    const int64_t np = L.pair_base[L.nbox];
    reserve_mapped(L.pr_slot, np);
    L.pr_slot.assign(np, -1);
    reserve_mapped(L.pr_t, (size_t)3 * np);
    L.pr_t.assign((size_t)3 * np, 0.0);
    reserve_mapped(L.pr_g, (size_t)2 * np);
    L.pr_g.assign((size_t)2 * np, 0.0);
    const double kappa = hp.kappa;
    const double inv4pi = 1.0 / (4.0 * kPi);
    parallel_for(L.nbox, [&](int64_t T) {
        const int64_t nT = L.box_start[T + 1] - L.box_start[T];
        for (int32_t c = L.cou_start[T]; c < L.cou_start[T + 1]; ++c) {
            const int32_t k = L.cou[c];
            const double* ctr = &L.box_ctr[3 * k];
            for (int64_t t = 0; t < nT; ++t) {
                const int64_t j = L.box_start[T] + t;
                ConeLoc cl;
                cone_locate(hp.pts[3 * j] - ctr[0], hp.pts[3 * j + 1] - ctr[1], hp.pts[3 * j + 2] - ctr[2], L.h, L.ds,
                            L.dang, L.ns, L.nc, cl);
                const int64_t e = L.pair_base[T] + (int64_t)(c - L.cou_start[T]) * nT + t;
                L.pr_slot[e] = host_lookup(L, k, cl.cell, cl.is);
                L.pr_t[e] = cl.ts;
                L.pr_t[np + e] = cl.tt;
                L.pr_t[2 * np + e] = cl.tp;
                // G(x, x_k) = e^{i k r} / (4 pi r)
                L.pr_g[e] = std::cos(kappa * cl.r) * inv4pi / cl.r;
                L.pr_g[np + e] = std::sin(kappa * cl.r) * inv4pi / cl.r;
            }
        }
    }, 1);
    L.use_pairs = true;
}

// The pairs with a cone, ordered by cone slot (stable: by target box, cousin
// and target), with a copy of their slot, local coordinates and centred
// factor in that order, for the two-phase evaluation.  Each slot's run is
// padded to a multiple of kPairQuad with placeholder entries (place -1, the
// slot's own cone, coordinates 0, factor 0), so that kPairQuad consecutive
// entries always share a cone.
void build_pair_order(HostLevel& L)
{
    const int64_t np = (int64_t)L.pr_slot.size();
    std::vector<int64_t> cnt((size_t)L.nslots, 0);
    for (int64_t e = 0; e < np; ++e)
        if (L.pr_slot[e] >= 0) cnt[(size_t)L.pr_slot[e]]++;
    std::vector<int64_t> start((size_t)L.nslots + 1, 0);
    for (int64_t s = 0; s < L.nslots; ++s)
        start[(size_t)s + 1] = start[(size_t)s] + (cnt[(size_t)s] + kPairQuad - 1) / kPairQuad * kPairQuad;
    const int64_t no = start[(size_t)L.nslots];
    reserve_mapped(L.pr_order, (size_t)no);
    L.pr_order.assign((size_t)no, -1);
    reserve_mapped(L.pro_slot, (size_t)no);
    L.pro_slot.assign((size_t)no, 0);
    for (int64_t s = 0; s < L.nslots; ++s)
        for (int64_t i = start[(size_t)s]; i < start[(size_t)s + 1]; ++i) L.pro_slot[(size_t)i] = (int32_t)s;
    {
        std::vector<int64_t> pos(start.begin(), start.end() - 1);
        for (int64_t e = 0; e < np; ++e)
            if (L.pr_slot[e] >= 0) L.pr_order[(size_t)pos[(size_t)L.pr_slot[e]]++] = (int32_t)e;
    }
    reserve_mapped(L.pro_t, (size_t)3 * no);
    L.pro_t.assign((size_t)3 * no, 0.0);
    reserve_mapped(L.pro_g, (size_t)2 * no);
    L.pro_g.assign((size_t)2 * no, 0.0);
    parallel_for(no, [&](int64_t i) {
        const int64_t e = L.pr_order[(size_t)i];
        if (e < 0) return;
        for (int c = 0; c < 3; ++c) L.pro_t[(size_t)c * no + i] = L.pr_t[(size_t)c * np + e];
        for (int c = 0; c < 2; ++c) L.pro_g[(size_t)c * no + i] = L.pr_g[(size_t)c * np + e];
    }, 4096);
}

// Parent boxes per block of the box tiles (IFGF_TILE_BLOCK overrides).
int64_t tile_box_block()
{
    const char* e = std::getenv("IFGF_TILE_BLOCK");
    const int64_t v = e ? std::atoll(e) : 16384;
    return v < 1 ? 1 : v;
}

// Whether the boxes of one cone are ordered by child mask before they are cut
// into tiles (IFGF_TILE_SORT=0 keeps Morton order).
int tile_sort()
{
    const char* e = std::getenv("IFGF_TILE_SORT");
    return e ? std::atoi(e) : 2;
}

// Device bytes a level's frame table may take when its frames are not shared
// (IFGF_FRAME_BUDGET_MB, default 3072).  IFGF_NO_FRAMES=1 disables the
// tables (the kernels then compute every geometry themselves).
double frame_budget_bytes()
{
    const char* e = std::getenv("IFGF_FRAME_BUDGET_MB");
    double mb = e ? std::atof(e) : 3072.0;
    return mb * 1024.0 * 1024.0;
}

// Child-to-parent frames of level d (children at d, parents at d - 1):
// every (parent slot, child) pair is described by (parent cone, child
// octant); the distinct pairs are tabulated once when they are shared at
// least four times on average or the table fits the frame budget, otherwise
// the kernels compute the geometry.
void build_frames(HostPlan& hp, int d)
{
    HostLevel& L = hp.L[d];
    const HostLevel& Lp = hp.L[d - 1];
    const int P = hp.P, ps = hp.ps, pang = hp.pang;
    reserve_mapped(L.child_of, (size_t)Lp.nbox * 8);
    L.child_of.assign((size_t)Lp.nbox * 8, -1);
    for (int64_t k = 0; k < L.nbox; ++k)
        if (L.active[k]) L.child_of[(size_t)L.parent[k] * 8 + L.box_oct[k]] = (int32_t)k;
    // the distinct (parent cone, octant) keys in increasing order: marked in a
    // bit set over the key space and read back in order (a sort where that
    // space is too large for one)
    const uint64_t kspace = (uint64_t)Lp.ncell * (uint64_t)Lp.ns * 8u;
    const bool bitset = kspace <= ((uint64_t)1 << 33);
    std::vector<uint64_t> keys;
    std::vector<uint64_t> kbits;
    std::vector<int64_t> kbase;
    if (bitset) {
        const int64_t nw = (int64_t)((kspace + 63) / 64);
        kbits.assign((size_t)nw, 0);
        parallel_for(Lp.nslots, [&](int64_t sl) {
            const int32_t j = Lp.slot_box[sl];
            for (int o = 0; o < 8; ++o)
                if (L.child_of[(size_t)j * 8 + o] >= 0) {
                    const uint64_t key = (uint64_t)Lp.slot_cone[sl] * 8 + o;
                    uint64_t* w = &kbits[key >> 6];
                    const uint64_t bit = 1ull << (key & 63);
                    // most keys recur: set a bit only where it is still clear
                    // (a read leaves the word shared between the threads)
                    if (!(__atomic_load_n(w, __ATOMIC_RELAXED) & bit)) __atomic_fetch_or(w, bit, __ATOMIC_RELAXED);
                }
        }, 1024);
        // every slot of box j pairs with each of j's children
        int64_t np = 0;
        for (int64_t j = 0; j < Lp.nbox; ++j) {
            int c = 0;
            for (int o = 0; o < 8; ++o) c += L.child_of[(size_t)j * 8 + o] >= 0;
            np += (int64_t)c * (Lp.slot_start[j + 1] - Lp.slot_start[j]);
        }
        L.npairs = np;
        kbase.assign((size_t)nw + 1, 0);
        for (int64_t w = 0; w < nw; ++w) kbase[w + 1] = kbase[w] + __builtin_popcountll(kbits[w]);
        keys.resize((size_t)kbase[nw]);
        parallel_for(nw, [&](int64_t w) {
            uint64_t m = kbits[w];
            int64_t i = kbase[w];
            while (m) {
                const int b = __builtin_ctzll(m);
                keys[(size_t)i++] = (uint64_t)w * 64 + (uint64_t)b;
                m &= m - 1;
            }
        }, 4096);
    } else {
        keys.reserve((size_t)Lp.nslots * 4);
        for (int64_t sl = 0; sl < Lp.nslots; ++sl) {
            int32_t j = Lp.slot_box[sl];
            for (int o = 0; o < 8; ++o)
                if (L.child_of[(size_t)j * 8 + o] >= 0) keys.push_back((uint64_t)Lp.slot_cone[sl] * 8 + o);
        }
        L.npairs = (int64_t)keys.size();
        parallel_sort(keys);
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    }
    L.nframes = (int64_t)keys.size();
    g_clock.lap("    frame keys");
    // tabulate when frames are shared at least 4x, or when the table is small
    // enough (it replaces FP64 geometry in the kernels, also at levels where
    // every frame is used once)
    const double budget = frame_budget_bytes();
    const char* nf = std::getenv("IFGF_NO_FRAMES");
    L.use_frames = !(nf && std::atoi(nf) != 0) &&
                   (L.nframes * 4 <= L.npairs || (double)L.nframes * P * 26.0 <= budget);
    if (!L.use_frames) {
        L.nframes = 0;
        return;
    }
    reserve_mapped(L.pframe, (size_t)Lp.nslots * 8);
    L.pframe.assign((size_t)Lp.nslots * 8, -1);
    parallel_for(Lp.nslots, [&](int64_t sl) {
        int32_t j = Lp.slot_box[sl];
        for (int o = 0; o < 8; ++o)
            if (L.child_of[(size_t)j * 8 + o] >= 0) {
                uint64_t key = (uint64_t)Lp.slot_cone[sl] * 8 + o;
                // the key's rank among the distinct keys
                L.pframe[(size_t)sl * 8 + o] =
                    bitset ? (int32_t)(kbase[key >> 6] +
                                       __builtin_popcountll(kbits[key >> 6] & ((1ull << (key & 63)) - 1ull)))
                           : (int32_t)(std::lower_bound(keys.begin(), keys.end(), key) - keys.begin());
            }
    }, 1024);
    g_clock.lap("    frame of each slot");
    reserve_mapped(L.fr_key, (size_t)L.nframes * P);
    L.fr_key.resize((size_t)L.nframes * P);
    reserve_mapped(L.fr_t, (size_t)L.nframes * P * 3);
    L.fr_t.resize((size_t)L.nframes * P * 3);
    reserve_mapped(L.fr_ratio, (size_t)L.nframes * P * 2);
    L.fr_ratio.resize((size_t)L.nframes * P * 2);
    const double kappa = hp.kappa;
    parallel_for(L.nframes, [&](int64_t f) {
        int64_t pc = (int64_t)(keys[f] >> 3);
        int oct = (int)(keys[f] & 7);
        double o[3];
        for (int a = 0; a < 3; ++a) o[a] = ((oct >> a) & 1) ? 0.5 * L.H : -0.5 * L.H;
        int pcell = (int)(pc / Lp.ns), pis = (int)(pc % Lp.ns);
        for (int a = 0; a < ps; ++a) {
            double rr = Lp.node_r[(size_t)pis * ps + a];
            for (int bb = 0; bb < pang; ++bb)
                for (int cc = 0; cc < pang; ++cc) {
                    int nu = (a * pang + bb) * pang + cc;
                    const double* dir = &Lp.node_dir[(((size_t)pcell * pang + bb) * pang + cc) * 3];
                    double v[3];
                    node_minus(rr, dir, o, v);
                    ConeLoc cl;
                    cone_locate(v[0], v[1], v[2], L.h, L.ds, L.dang, L.ns, L.nc, cl);
                    size_t e = (size_t)f * P + nu;
                    L.fr_key[e] = (uint32_t)((int64_t)cl.cell * L.ns + cl.is);
                    L.fr_t[3 * e] = cl.ts;
                    L.fr_t[3 * e + 1] = cl.tt;
                    L.fr_t[3 * e + 2] = cl.tp;
                    // G(x, x_k) / G(x, x_j) = |y| / |y - o| e^{i k (|y - o| - |y|)},
                    // |y - o| - |y| = (|o|^2 - 2 y.o) / (|y - o| + |y|), y = x - x_j
                    double y[3] = {rr * dir[0], rr * dir[1], rr * dir[2]};
                    double ry = std::sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                    double num = (o[0] * o[0] + o[1] * o[1] + o[2] * o[2]) - 2.0 * (y[0] * o[0] + y[1] * o[1] + y[2] * o[2]);
                    double diff = num / (cl.r + ry);
                    double mag = ry / cl.r;
                    L.fr_ratio[2 * e] = mag * std::cos(kappa * diff);
                    L.fr_ratio[2 * e + 1] = mag * std::sin(kappa * diff);
                }
        }
    }, 64);
    g_clock.lap("    frame geometry");
    // groups: distinct child cones per frame, in order of first appearance
    L.fr_ngrp.assign(L.nframes, 0);
    reserve_mapped(L.fr_gkey, (size_t)L.nframes * kMaxFrameGroups);
    L.fr_gkey.assign((size_t)L.nframes * kMaxFrameGroups, 0);
    reserve_mapped(L.fr_grp, (size_t)L.nframes * P);
    L.fr_grp.assign((size_t)L.nframes * P, 0);
    std::atomic<int> too_many{0};
    parallel_for(L.nframes, [&](int64_t f) {
        int ng = 0;
        uint32_t* gk = &L.fr_gkey[(size_t)f * kMaxFrameGroups];
        for (int nu = 0; nu < P; ++nu) {
            uint32_t key = L.fr_key[(size_t)f * P + nu];
            int g = 0;
            while (g < ng && gk[g] != key) ++g;
            if (g == ng) {
                if (ng == kMaxFrameGroups) {
                    too_many = 1;
                    return;
                }
                gk[ng++] = key;
            }
            L.fr_grp[(size_t)f * P + nu] = (uint8_t)g;
        }
        L.fr_ngrp[f] = (uint8_t)ng;
    }, 256);
    L.frame_groups_ok = too_many.load() == 0 && P <= 255;
    L.fr_max_groups = 0;
    for (int64_t f = 0; f < L.nframes; ++f) L.fr_max_groups = std::max<int>(L.fr_max_groups, L.fr_ngrp[f]);
    if (!L.frame_groups_ok) return;
    // the points of each frame ordered by group (for tiles of one child cone)
    reserve_mapped(L.fr_order, (size_t)L.nframes * P);
    L.fr_order.assign((size_t)L.nframes * P, 0);
    L.fr_goff.assign((size_t)L.nframes * (kMaxFrameGroups + 1), 0);
    parallel_for(L.nframes, [&](int64_t f) {
        const uint8_t* grp = &L.fr_grp[(size_t)f * P];
        uint8_t* off = &L.fr_goff[(size_t)f * (kMaxFrameGroups + 1)];
        int ng = L.fr_ngrp[f];
        int cnt[kMaxFrameGroups + 1] = {0};
        for (int nu = 0; nu < P; ++nu) cnt[grp[nu] + 1]++;
        for (int g = 0; g < ng; ++g) cnt[g + 1] += cnt[g];
        for (int g = 0; g <= ng; ++g) off[g] = (uint8_t)cnt[g];
        for (int g = ng + 1; g <= kMaxFrameGroups; ++g) off[g] = (uint8_t)P;
        uint8_t* ord = &L.fr_order[(size_t)f * P];
        for (int nu = 0; nu < P; ++nu) ord[cnt[grp[nu]]++] = (uint8_t)nu;
    }, 256);
    // box tiles.  The parent boxes are cut into blocks of consecutive
    // (Morton-ordered) boxes; within a block the slots are sorted by cone,
    // then by the mask of children their box has, and every run of one cone
    // is cut into tiles.  A tile runs one pass per octant that any of its
    // boxes has a child in, so boxes with the same children in one tile
    // leave fewer columns of those passes empty (near a surface a box has 3-4
    // of its 8 children).  Large blocks give long runs, hence full tiles of
    // like masks; small blocks keep the child cones a block reads together
    // in cache.
    g_clock.lap("    frame groups");
    const int64_t blk = tile_box_block();
    const int64_t nblk = (Lp.nbox + blk - 1) / blk;
    const int mode = tile_sort();
    std::vector<std::vector<int32_t>> btiles(nblk);   // kBoxTile entries per tile, -1 padded
    std::vector<int64_t> bt(nblk + 1, 0);
    struct SlotKey {
        uint64_t k;   // parent cone << 8 | child mask (0 in mode 0)
        int32_t s;    // slot, which breaks ties in the order of the slots
    };
    // a run's tiles as kBoxTile entries each (-1 padded); cost = the octant
    // passes they run
    auto emit = [](std::vector<int32_t>& dst, const int32_t* sl, int n) {
        for (int k = 0; k < kBoxTile; ++k) dst.push_back(k < n ? sl[k] : -1);
    };
    struct Open {
        int m, n;
        int32_t s[kBoxTile];
    };
    // blocks one after the other, each block's sort and runs on all threads
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t j0 = b * blk, j1 = std::min<int64_t>(Lp.nbox, j0 + blk);
        const int32_t s0 = Lp.slot_start[j0];
        const int64_t nsb = Lp.slot_start[j1] - s0;
        // the children of each box of the block (bit o: a child in octant o)
        std::vector<uint8_t> bm((size_t)(j1 - j0));
        parallel_for(j1 - j0, [&](int64_t j) {
            int m = 0;
            for (int o = 0; o < 8; ++o) m |= (L.child_of[(size_t)(j0 + j) * 8 + o] >= 0) << o;
            bm[j] = (uint8_t)m;
        }, 1024);
        auto mask = [&](int32_t sl) { return (int)bm[Lp.slot_box[sl] - j0]; };
        // the block's slots by parent cone, then (unless mode 0) child mask,
        // in slot order among equals
        std::vector<int32_t> v((size_t)nsb);
        const int64_t ncone = (int64_t)Lp.ncell * Lp.ns;
        const int nch = host_threads();
        if (ncone * nch <= ((int64_t)1 << 24)) {
            // two stable counting sorts over nch chunks (a histogram per
            // chunk): by child mask (unless mode 0), then by cone
            std::vector<int64_t> hist((size_t)(nch * std::max<int64_t>(ncone, 256)));
            auto csort = [&](const int32_t* src, int32_t* dst, int64_t nkey, auto&& key) {
                std::fill(hist.begin(), hist.begin() + nch * nkey, 0);
                parallel_for(nch, [&](int64_t c) {
                    int64_t* hc = &hist[(size_t)(c * nkey)];
                    for (int64_t i = nsb * c / nch; i < nsb * (c + 1) / nch; ++i) hc[key(src[i])]++;
                });
                int64_t off = 0;
                for (int64_t q = 0; q < nkey; ++q)
                    for (int c = 0; c < nch; ++c) {
                        const int64_t t = hist[(size_t)(c * nkey + q)];
                        hist[(size_t)(c * nkey + q)] = off;
                        off += t;
                    }
                parallel_for(nch, [&](int64_t c) {
                    int64_t* hc = &hist[(size_t)(c * nkey)];
                    for (int64_t i = nsb * c / nch; i < nsb * (c + 1) / nch; ++i) dst[hc[key(src[i])]++] = src[i];
                });
            };
            std::vector<int32_t> w((size_t)nsb);
            std::iota(w.begin(), w.end(), s0);
            if (mode != 0) {
                csort(w.data(), v.data(), 256, [&](int32_t sl) { return mask(sl); });
                w.swap(v);
            }
            csort(w.data(), v.data(), ncone, [&](int32_t sl) { return (int64_t)Lp.slot_cone[sl]; });
        } else {
            std::vector<SlotKey> sk((size_t)nsb);
            parallel_for(nsb, [&](int64_t i) {
                const int32_t sl = s0 + (int32_t)i;
                sk[i] = SlotKey{((uint64_t)(uint32_t)Lp.slot_cone[sl] << 8) | (uint64_t)(mode != 0 ? mask(sl) : 0), sl};
            }, 4096);
            parallel_stable_sort(sk, [](const SlotKey& x, const SlotKey& y) { return x.k != y.k ? x.k < y.k : x.s < y.s; });
            parallel_for(nsb, [&](int64_t k) { v[k] = sk[k].s; }, 4096);
        }
        std::vector<int> mk((size_t)nsb);
        parallel_for(nsb, [&](int64_t k) { mk[k] = mask(v[k]); }, 4096);
        // runs of one parent cone
        std::vector<size_t> run{0};
        for (size_t k = 1; k < v.size(); ++k)
            if (Lp.slot_cone[v[k]] != Lp.slot_cone[v[k - 1]]) run.push_back(k);
        run.push_back(v.size());
        const int64_t nrun = (int64_t)run.size() - 1;
        std::vector<std::vector<int32_t>> rout(nrun);
        parallel_for(nrun, [&](int64_t r) {
            const size_t i = run[r], e = run[r + 1];
            auto cost = [&](const std::vector<int32_t>& w) {
                int64_t c = 0;
                for (size_t t = 0; t < w.size(); t += kBoxTile) {
                    int m = 0;
                    for (int k = 0; k < kBoxTile; ++k)
                        if (w[t + k] >= 0) m |= mask(w[t + k]);
                    c += __builtin_popcount(m);
                }
                return c;
            };
            // the run cut in order (by child mask unless mode 0)
            std::vector<int32_t> cut;
            for (size_t k0 = i; k0 < e; k0 += kBoxTile) emit(cut, &v[k0], (int)std::min<size_t>(kBoxTile, e - k0));
            if (mode != 2 || e - i <= (size_t)kBoxTile) {
                rout[r].swap(cut);
                return;
            }
            // or: full tiles of one child mask, then the rest, largest masks
            // first, each to the open tile whose octants it widens least;
            // the run keeps whichever of the two runs fewer passes
            std::vector<int32_t> grp;
            std::vector<size_t> rem;
            for (size_t a = i; a < e;) {
                size_t z = a;
                while (z < e && mk[z] == mk[a]) ++z;
                size_t a1 = a;
                for (; a1 + kBoxTile <= z; a1 += kBoxTile) emit(grp, &v[a1], kBoxTile);
                for (; a1 < z; ++a1) rem.push_back(a1);
                a = z;
            }
            std::stable_sort(rem.begin(), rem.end(), [&](size_t x, size_t y) {
                return __builtin_popcount(mk[x]) > __builtin_popcount(mk[y]);
            });
            std::vector<Open> open;
            for (size_t x : rem) {
                int best = -1, bg = 9;
                for (int t = 0; t < (int)open.size(); ++t) {
                    if (open[t].n == kBoxTile) continue;
                    const int g = __builtin_popcount(open[t].m | mk[x]) - __builtin_popcount(open[t].m);
                    if (g < bg || (g == bg && open[t].n > open[best].n)) {
                        best = t;
                        bg = g;
                    }
                }
                if (best < 0) {
                    open.push_back(Open{0, 0, {}});
                    best = (int)open.size() - 1;
                }
                open[best].m |= mk[x];
                open[best].s[open[best].n++] = v[x];
            }
            for (const Open& t : open) emit(grp, t.s, t.n);
            if (cost(grp) < cost(cut)) rout[r].swap(grp);
            else rout[r].swap(cut);
        }, 64);
        std::vector<int32_t>& out = btiles[b];
        size_t tot = 0;
        for (const auto& w : rout) tot += w.size();
        out.reserve(tot);
        for (const auto& w : rout) out.insert(out.end(), w.begin(), w.end());
        bt[b + 1] = (int64_t)(out.size() / kBoxTile);
    }
    for (int64_t b = 0; b < nblk; ++b) bt[b + 1] += bt[b];
    L.ntiles = bt[nblk];
    reserve_mapped(L.bt_slot, (size_t)L.ntiles * kBoxTile);
    L.bt_slot.assign((size_t)L.ntiles * kBoxTile, -1);
    L.bt_frame.assign((size_t)L.ntiles * 8, -1);
    parallel_for(nblk, [&](int64_t b) {
        const std::vector<int32_t>& w = btiles[b];
        std::copy(w.begin(), w.end(), L.bt_slot.begin() + bt[b] * kBoxTile);
        for (int64_t t = bt[b]; t < bt[b + 1]; ++t)
            for (int k = 0; k < kBoxTile; ++k) {
                const int32_t sl = L.bt_slot[(size_t)t * kBoxTile + k];
                if (sl < 0) continue;
                for (int o = 0; o < 8; ++o)
                    if (L.pframe[(size_t)sl * 8 + o] >= 0) L.bt_frame[(size_t)t * 8 + o] = L.pframe[(size_t)sl * 8 + o];
            }
    }, 1);
    L.slot_order.clear();
    L.slot_order.reserve((size_t)Lp.nslots);
    for (int32_t sl : L.bt_slot)
        if (sl >= 0) L.slot_order.push_back(sl);
}

// The entries of level d's box tiles: for every tile, its frames' (octant,
// group) pairs in octant order, each with the child slot it reads in each of
// the tile's boxes, so that a tile's kernel reads them in one step instead of
// looking up frames, children and cones one after the other.
void build_tile_entries(HostPlan& hp, int d)
{
    HostLevel& L = hp.L[d];
    const HostLevel& Lp = hp.L[d - 1];
    constexpr int G = kMaxFrameGroups;
    const int64_t nt = L.ntiles;
    L.te_start.assign(nt + 1, 0);
    for (int64_t t = 0; t < nt; ++t) {
        int n = 0;
        for (int o = 0; o < 8; ++o) {
            const int32_t f = L.bt_frame[(size_t)t * 8 + o];
            if (f >= 0) n += L.fr_ngrp[f];
        }
        L.te_start[t + 1] = L.te_start[t] + n;
    }
    const int64_t ne = L.te_start[nt];
    L.te_per_tile = nt > 0 ? (double)ne / (double)nt : 0.0;
    L.te_go.assign((size_t)nt * 9, 0);
    L.te_mask.assign((size_t)nt * kBoxTile, 0);
    reserve_mapped(L.te_info, (size_t)ne);
    L.te_info.assign((size_t)ne, 0);
    reserve_mapped(L.te_cs, (size_t)ne * kBoxTile);
    L.te_cs.assign((size_t)ne * kBoxTile, -1);
    parallel_for(nt, [&](int64_t t) {
        int32_t kid[kBoxTile][8];
        for (int bi = 0; bi < kBoxTile; ++bi) {
            const int32_t sl = L.bt_slot[(size_t)t * kBoxTile + bi];
            int m = 0;
            for (int o = 0; o < 8; ++o) {
                kid[bi][o] = sl >= 0 ? L.child_of[(size_t)Lp.slot_box[sl] * 8 + o] : -1;
                m |= (kid[bi][o] >= 0) << o;
            }
            L.te_mask[(size_t)t * kBoxTile + bi] = (uint8_t)m;
        }
        int64_t e = L.te_start[t];
        for (int o = 0; o < 8; ++o) {
            L.te_go[(size_t)t * 9 + o] = (uint16_t)(e - L.te_start[t]);
            const int32_t f = L.bt_frame[(size_t)t * 8 + o];
            if (f < 0) continue;
            for (int g = 0; g < L.fr_ngrp[f]; ++g, ++e) {
                const int g0 = L.fr_goff[(size_t)f * (G + 1) + g], g1 = L.fr_goff[(size_t)f * (G + 1) + g + 1];
                L.te_info[e] = g0 | ((g1 - g0) << 8) | (o << 16);
                const uint32_t key = L.fr_gkey[(size_t)f * G + g];
                const int cell = (int)(key / (uint32_t)L.ns), is = (int)(key - (uint32_t)cell * L.ns);
                for (int bi = 0; bi < kBoxTile; ++bi) {
                    const int32_t k = kid[bi][o];
                    int32_t cs = -1;
                    if (k >= 0) {
                        cs = host_lookup(L, k, cell, is);
                        if (cs < 0) cs = -2;
                    }
                    L.te_cs[(size_t)e * kBoxTile + bi] = cs;
                }
            }
        }
        L.te_go[(size_t)t * 9 + 8] = (uint16_t)(e - L.te_start[t]);
    }, 64);
}

}  // namespace

std::string build_host_plan(const double* points, int64_t n, double kappa, int levels, int ps, int pang,
                            int leaf_ns, int leaf_nc, bool dilate, double tab_elem_bytes, double ord_elem_bytes,
                            double pair_budget, HostPlan& hp, ifgf_status& code, ConeMarker* marker,
                            bool pairs_device, int leaf_max)
{
    auto t0 = std::chrono::steady_clock::now();
    g_clock.start();
    auto phase = [&](const char* what) { g_clock.lap(what); };
    code = IFGF_E_INVALID_ARG;
    if (!points) return "points is NULL";
    if (n < 2) return "need at least two points";
    if (n > (int64_t)INT32_MAX / 2) return "too many points for 32-bit indexing";
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) return "wavenumber must be finite and >= 0";
    if (levels < 0 || levels > 22) return "levels must be 0 (auto) or 2..22";
    if (levels == 1) return "levels must be 0 (auto) or 2..22";
    if (leaf_ns < 1 || leaf_nc < 1 || leaf_ns > 64 || leaf_nc > 64) return "leaf cone counts out of range";
    if (leaf_max < 0) return "leaf_max must be >= 0";
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(points[i])) return "points must be finite";

    hp = HostPlan();
    hp.n = n;
    hp.kappa = kappa;
    hp.ps = ps;
    hp.pang = pang;
    hp.P = ps * pang * pang;

    // Root box: centre at the bounding-box midpoint, side = largest extent.
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = points[a];
    for (int64_t i = 1; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], points[3 * i + a]);
            hi[a] = std::max(hi[a], points[3 * i + a]);
        }
    double H1 = 0.0;
    for (int a = 0; a < 3; ++a) {
        hp.x1[a] = 0.5 * (lo[a] + hi[a]);
        H1 = std::max(H1, hi[a] - lo[a]);
    }
    if (!(H1 > 0.0)) return "all points coincide";
    hp.H1 = H1;
    for (int a = 0; a < 3; ++a) hp.corner[a] = hp.x1[a] - H1 / 2.0;

    // Number of levels: leaf boxes about a quarter wavelength wide (Sec. 4).
    int D = levels;
    if (D == 0) {
        if (kappa > 0.0) {
            double lambda = 2.0 * kPi / kappa;
            D = 1 + (int)std::floor(std::log2(4.0 * H1 / lambda) + 0.5);
        } else {
            for (D = 2; D < 22; ++D) {
                double Hd = std::ldexp(H1, -(D - 1));
                int64_t nb = (int64_t)1 << (D - 1);
                std::vector<uint64_t> keys(n);
                for (int64_t i = 0; i < n; ++i) {
                    int64_t k[3];
                    box_index(&points[3 * i], hp.corner, Hd, nb, k);
                    keys[i] = ((uint64_t)k[0] << 42) | ((uint64_t)k[1] << 21) | (uint64_t)k[2];
                }
                std::sort(keys.begin(), keys.end());
                int64_t nu = std::unique(keys.begin(), keys.end()) - keys.begin();
                if ((double)n / (double)nu <= 8.0) break;
            }
        }
        D = std::max(2, std::min(22, D));
    }
    hp.D = D;
    const int bits = D - 1;
    const double HD = std::ldexp(H1, -(D - 1));
    const int64_t nbD = (int64_t)1 << (D - 1);

    phase("root box and levels");
    // Leaf multi-index and Morton code of every point; sort by code (ties by
    // coordinates, so equal points become neighbours in the order).
    std::vector<int64_t> kD(3 * n);
    std::vector<uint64_t> mort(n);
    parallel_for(n, [&](int64_t i) {
        box_index(&points[3 * i], hp.corner, HD, nbD, &kD[3 * i]);
        mort[i] = interleave3(kD[3 * i], kD[3 * i + 1], kD[3 * i + 2], bits);
    }, 4096);
    // (code, point) pairs sorted on the thread pool; the order is total, so
    // the permutation is the one any sort gives
    struct MortonKey {
        uint64_t code;
        int32_t i;
    };
    std::vector<MortonKey> mo((size_t)n);
    parallel_for(n, [&](int64_t i) { mo[i] = MortonKey{mort[i], (int32_t)i}; }, 4096);
    parallel_stable_sort(mo, [&](const MortonKey& x, const MortonKey& y) {
        if (x.code != y.code) return x.code < y.code;
        for (int c = 0; c < 3; ++c)
            if (points[3 * x.i + c] != points[3 * y.i + c]) return points[3 * x.i + c] < points[3 * y.i + c];
        return x.i < y.i;
    });
    std::vector<int32_t> order(n);
    parallel_for(n, [&](int64_t i) { order[i] = mo[i].i; }, 4096);
    std::vector<MortonKey>().swap(mo);
    for (int64_t i = 1; i < n; ++i) {
        int32_t a = order[i - 1], b = order[i];
        if (mort[a] == mort[b] && points[3 * a] == points[3 * b] && points[3 * a + 1] == points[3 * b + 1] &&
            points[3 * a + 2] == points[3 * b + 2])
            return "points must be pairwise different (duplicates of input point " + std::to_string(a) + ")";
    }
    hp.perm = order;
    hp.pts.resize(3 * n);
    std::vector<uint64_t> mcode(n);
    std::vector<int64_t> mk(3 * n);
    parallel_for(n, [&](int64_t i) {
        for (int a = 0; a < 3; ++a) {
            hp.pts[3 * i + a] = points[3 * order[i] + a];
            mk[3 * i + a] = kD[3 * order[i] + a];
        }
        mcode[i] = mort[order[i]];
    }, 4096);

    phase("Morton sort");
    // Relevant boxes of every level: unique Morton prefixes.
    hp.L.assign(D + 1, HostLevel());
    for (int d = 1; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        L.H = std::ldexp(H1, -(d - 1));
        L.h = std::sqrt(3.0) * L.H / 2.0;
        int shift = 3 * (D - d);
        L.pt_box.resize(n);
        for (int64_t i = 0; i < n; ++i) {
            uint64_t p = mcode[i] >> shift;
            if (i == 0 || p != L.prefix.back()) {
                L.prefix.push_back(p);
                L.box_start.push_back((int32_t)i);
            }
            L.pt_box[i] = (int32_t)L.prefix.size() - 1;
        }
        L.nbox = (int64_t)L.prefix.size();
        L.box_start.push_back((int32_t)n);
        L.box_ctr.resize(3 * L.nbox);
        L.box_oct.resize(L.nbox);
        for (int64_t b = 0; b < L.nbox; ++b) {
            int64_t i = L.box_start[b];
            int64_t k[3];
            for (int a = 0; a < 3; ++a) k[a] = mk[3 * i + a] >> (D - d);
            // x_k^d = x_1^1 - H_1/2 + H_d/2 (2k - 1), 1-based k (eq. defboxsizesandcenters)
            for (int a = 0; a < 3; ++a) L.box_ctr[3 * b + a] = hp.x1[a] - H1 / 2.0 + L.H / 2.0 * (2.0 * k[a] + 1.0);
            L.box_oct[b] = (uint8_t)((k[0] & 1) | ((k[1] & 1) << 1) | ((k[2] & 1) << 2));
        }
    }

    phase("relevant boxes");
    // Parents and children.
    for (int d = 1; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        L.parent.assign(L.nbox, -1);
        if (d > 1) {
            const HostLevel& Lp = hp.L[d - 1];
            int64_t p = 0;
            for (int64_t b = 0; b < L.nbox; ++b) {
                uint64_t pk = L.prefix[b] >> 3;
                while (Lp.prefix[p] != pk) ++p;
                L.parent[b] = (int32_t)p;
            }
        }
    }
    for (int d = 1; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        L.chl_start.assign(L.nbox + 1, 0);
        if (d < D) {
            const HostLevel& Lc = hp.L[d + 1];
            for (int64_t c = 0; c < Lc.nbox; ++c) L.chl_start[Lc.parent[c] + 1]++;
            for (int64_t b = 0; b < L.nbox; ++b) L.chl_start[b + 1] += L.chl_start[b];
            L.chl.resize(Lc.nbox);
            for (int64_t c = 0; c < Lc.nbox; ++c) L.chl[c] = (int32_t)c;  // children are contiguous and ordered
        }
    }

    // The source tree (adaptive octree): the root is split; below it a box is
    // active when its parent is active and not a leaf, and an active box is a
    // leaf on level D or when it holds at most leaf_max points.
    hp.leaf_max = leaf_max;
    hp.adaptive = false;
    for (int d = 1; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        L.active.assign(L.nbox, 0);
        L.leaf.assign(L.nbox, 0);
        for (int64_t b = 0; b < L.nbox; ++b) {
            if (d == 1) {
                L.active[b] = 1;
                continue;
            }
            const HostLevel& Lp = hp.L[d - 1];
            const int32_t p = L.parent[b];
            L.active[b] = Lp.active[p] && !Lp.leaf[p];
            const int64_t cnt = L.box_start[b + 1] - L.box_start[b];
            L.leaf[b] = L.active[b] && (d == D || (leaf_max > 0 && cnt <= leaf_max));
            if (L.leaf[b] && d < D) hp.adaptive = true;
        }
    }

    phase("parents and children");
    // Neighbours (|a - k|_inf <= 1, self included) on every level.
    for (int d = 1; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        int64_t nb = (int64_t)1 << (d - 1);
        std::vector<int32_t> cnt(L.nbox), tmp(27 * L.nbox);
        parallel_for(L.nbox, [&](int64_t b) {
            int64_t k[3];
            deinterleave3(L.prefix[b], d - 1, k);
            int c = 0;
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int64_t q[3] = {k[0] + dx, k[1] + dy, k[2] + dz};
                        if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= nb || q[1] >= nb || q[2] >= nb) continue;
                        int64_t j = find_prefix(L.prefix, interleave3(q[0], q[1], q[2], d - 1));
                        if (j >= 0) tmp[27 * b + c++] = (int32_t)j;
                    }
            std::sort(&tmp[27 * b], &tmp[27 * b] + c);
            cnt[b] = c;
        }, 256);
        L.nbr_start.assign(L.nbox + 1, 0);
        for (int64_t b = 0; b < L.nbox; ++b) L.nbr_start[b + 1] = L.nbr_start[b] + cnt[b];
        L.nbr.resize(L.nbr_start[L.nbox]);
        for (int64_t b = 0; b < L.nbox; ++b)
            std::copy(&tmp[27 * b], &tmp[27 * b] + cnt[b], &L.nbr[L.nbr_start[b]]);
    }

    phase("neighbours");
    // Cousins: relevant children of the parent's neighbours that are not
    // neighbours themselves (eq. defcousinboxes).
    for (int d = 1; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        L.cou_start.assign(L.nbox + 1, 0);
        if (d < 3) continue;
        const HostLevel& Lp = hp.L[d - 1];
        // the cousins of box b, in order, to f
        auto each_cousin = [&](int64_t b, auto&& f) {
            int64_t k[3];
            deinterleave3(L.prefix[b], d - 1, k);
            int32_t p = L.parent[b];
            for (int32_t qi = Lp.nbr_start[p]; qi < Lp.nbr_start[p + 1]; ++qi) {
                int32_t q = Lp.nbr[qi];
                for (int32_t c = Lp.chl_start[q]; c < Lp.chl_start[q + 1]; ++c) {
                    int64_t kc[3];
                    deinterleave3(L.prefix[c], d - 1, kc);
                    if (std::llabs(kc[0] - k[0]) <= 1 && std::llabs(kc[1] - k[1]) <= 1 && std::llabs(kc[2] - k[2]) <= 1)
                        continue;
                    f((int32_t)c);
                }
            }
        };
        if (!hp.adaptive) {
            // counted, then written in place, both on the thread pool
            parallel_for(L.nbox, [&](int64_t b) {
                int32_t m = 0;
                each_cousin(b, [&](int32_t) { ++m; });
                L.cou_start[b + 1] = m;
            }, 64);
            for (int64_t b = 0; b < L.nbox; ++b) L.cou_start[b + 1] += L.cou_start[b];
            reserve_mapped(L.cou, (size_t)L.cou_start[L.nbox]);
            L.cou.resize(L.cou_start[L.nbox]);
            parallel_for(L.nbox, [&](int64_t b) {
                int32_t* o = L.cou.data() + L.cou_start[b];
                each_cousin(b, [&](int32_t c) { *o++ = c; });
            }, 64);
            continue;
        }
        std::vector<std::vector<int32_t>> lists(L.nbox);
        parallel_for(L.nbox, [&](int64_t b) { each_cousin(b, [&](int32_t c) { lists[b].push_back(c); }); }, 64);
        if (hp.adaptive) {
            // rule (i) of an active box reads all its cousins; the evaluation
            // at the targets of a box reads its cousins that are source boxes
            L.mcou_start.assign(L.nbox + 1, 0);
            for (int64_t b = 0; b < L.nbox; ++b)
                L.mcou_start[b + 1] = L.mcou_start[b] + (L.active[b] ? (int32_t)lists[b].size() : 0);
            L.mcou.resize(L.mcou_start[L.nbox]);
            for (int64_t b = 0; b < L.nbox; ++b)
                if (L.active[b]) std::copy(lists[b].begin(), lists[b].end(), &L.mcou[L.mcou_start[b]]);
            for (int64_t b = 0; b < L.nbox; ++b) {
                auto& v = lists[b];
                v.erase(std::remove_if(v.begin(), v.end(), [&](int32_t c) { return !L.active[c]; }), v.end());
            }
        }
        for (int64_t b = 0; b < L.nbox; ++b) L.cou_start[b + 1] = L.cou_start[b] + (int32_t)lists[b].size();
        L.cou.resize(L.cou_start[L.nbox]);
        for (int64_t b = 0; b < L.nbox; ++b) std::copy(lists[b].begin(), lists[b].end(), &L.cou[L.cou_start[b]]);
    }

    phase("cousins");
    // Cone intervals: leaf counts given; going up, a_d = 2 iff 2 kappa H_d > 1.
    hp.L[D].ns = leaf_ns;
    hp.L[D].nc = leaf_nc;
    for (int d = D; d >= 2; --d) {
        int ad = (2.0 * kappa * hp.L[d].H > 1.0) ? 2 : 1;
        hp.L[d - 1].ns = ad * hp.L[d].ns;
        hp.L[d - 1].nc = ad * hp.L[d].nc;
    }
    const ChebNodes cs = make_cheb_nodes(ps), ca = make_cheb_nodes(pang);
    const double eta = std::sqrt(3.0) / 3.0;
    for (int d = 1; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        if ((int64_t)L.ns * L.nc * 2 * L.nc > (int64_t)1 << 30) {
            code = IFGF_E_UNSUPPORTED;
            return "too many cone segments per box at level " + std::to_string(d);
        }
        L.ds = eta / L.ns;
        L.dang = kPi / L.nc;
        L.ncell = L.nc * 2 * L.nc;
        L.W = (L.ns + 63) / 64;
        if (d < 3) continue;
        // interpolation points (eq. interp_pts): radii h / s and unit directions
        L.node_r.resize((size_t)L.ns * ps);
        for (int is = 0; is < L.ns; ++is)
            for (int a = 0; a < ps; ++a) {
                double s = L.ds * (is + 0.5 * (cs.t[a] + 1.0));
                L.node_r[(size_t)is * ps + a] = L.h / s;
            }
        L.node_dir.resize((size_t)L.ncell * pang * pang * 3);
        for (int it = 0; it < L.nc; ++it)
            for (int ip = 0; ip < 2 * L.nc; ++ip)
                for (int b = 0; b < pang; ++b)
                    for (int c = 0; c < pang; ++c) {
                        double th = L.dang * (it + 0.5 * (ca.t[b] + 1.0));
                        double ph = L.dang * (ip + 0.5 * (ca.t[c] + 1.0));
                        size_t o = ((((size_t)it * 2 * L.nc + ip) * pang + b) * pang + c) * 3;
                        L.node_dir[o] = std::sin(th) * std::cos(ph);
                        L.node_dir[o + 1] = std::sin(th) * std::sin(ph);
                        L.node_dir[o + 2] = std::cos(th);
                    }
    }

    phase("cone intervals and nodes");
    // Relevant cone segments, sweeping d = 3..D (eq. defallrelevantconesegments):
    // (i) the cone of every cousin point, (ii) for d >= 4 the cone of every
    // interpolation point of the parent's relevant cones.
    int64_t n_dilated = 0;
    for (int d = 3; d <= D; ++d) {
        HostLevel& L = hp.L[d];
        const int64_t ncone = (int64_t)L.ncell * L.ns;
        const int64_t wpb = (ncone + 63) / 64;
        std::vector<uint64_t> prim((size_t)L.nbox * wpb, 0), dil;
        if (dilate) dil.assign((size_t)L.nbox * wpb, 0);
        const double tol = kDilateTol;
        auto mark = [&](int64_t b, const ConeLoc& c) {
            uint64_t* P = &prim[(size_t)b * wpb];
            int64_t bit = (int64_t)c.cell * L.ns + c.is;
            P[bit >> 6] |= 1ull << (bit & 63);
            if (!dilate) return;
            int ls[3] = {c.is, c.is, c.is}, lt[3] = {c.it, c.it, c.it}, lp[3] = {c.ip, c.ip, c.ip};
            int nsv = 1, ntv = 1, npv = 1;
            if (c.ts > 1.0 - tol && c.is + 1 < L.ns) ls[nsv++] = c.is + 1;
            if (c.ts < -1.0 + tol && c.is > 0) ls[nsv++] = c.is - 1;
            if (c.tt > 1.0 - tol && c.it + 1 < L.nc) lt[ntv++] = c.it + 1;
            if (c.tt < -1.0 + tol && c.it > 0) lt[ntv++] = c.it - 1;
            if (c.tp > 1.0 - tol) lp[npv++] = (c.ip + 1) % (2 * L.nc);
            if (c.tp < -1.0 + tol) lp[npv++] = (c.ip + 2 * L.nc - 1) % (2 * L.nc);
            if (nsv * ntv * npv == 1) return;
            uint64_t* Q = &dil[(size_t)b * wpb];
            for (int i = 0; i < nsv; ++i)
                for (int j = 0; j < ntv; ++j)
                    for (int k = 0; k < npv; ++k) {
                        int64_t cb = ((int64_t)lt[j] * 2 * L.nc + lp[k]) * L.ns + ls[i];
                        Q[cb >> 6] |= 1ull << (cb & 63);
                    }
        };
        const HostLevel* Lp = &hp.L[d - 1];
        if (d >= 4) {
            build_frames(hp, d);
            phase("  frames (level)");
        }
        if (marker) {
            std::string err = marker->mark_level(hp, d, dilate, n_dilated, code);
            if (!err.empty()) return err;
            phase("  relevant cones on the GPU (level)");
            continue;
        }
        const std::vector<int32_t>& mst = hp.adaptive ? L.mcou_start : L.cou_start;
        const std::vector<int32_t>& mco = hp.adaptive ? L.mcou : L.cou;
        parallel_for(L.nbox, [&](int64_t b) {
            if (!L.active[b]) return;   // not a source box: no cones
            const double* ctr = &L.box_ctr[3 * b];
            for (int32_t ci = mst[b]; ci < mst[b + 1]; ++ci) {
                int32_t c = mco[ci];
                for (int32_t j = L.box_start[c]; j < L.box_start[c + 1]; ++j) {
                    ConeLoc cl;
                    cone_locate(hp.pts[3 * j] - ctr[0], hp.pts[3 * j + 1] - ctr[1], hp.pts[3 * j + 2] - ctr[2], L.h,
                                L.ds, L.dang, L.ns, L.nc, cl);
                    mark(b, cl);
                }
            }
            if (d >= 4 && L.use_frames) {
                // (ii) through the frames: the same decisions the kernels use
                int32_t p = L.parent[b];
                int o = L.box_oct[b];
                for (int32_t sl = Lp->slot_start[p]; sl < Lp->slot_start[p + 1]; ++sl) {
                    int32_t f = L.pframe[(size_t)sl * 8 + o];
                    const uint32_t* key = &L.fr_key[(size_t)f * hp.P];
                    uint64_t* Pm = &prim[(size_t)b * wpb];
                    for (int nu = 0; nu < hp.P; ++nu) {
                        int64_t bit = key[nu];
                        Pm[bit >> 6] |= 1ull << (bit & 63);
                    }
                }
            } else if (d >= 4) {
                int32_t p = L.parent[b];
                double o[3];
                for (int a = 0; a < 3; ++a) o[a] = ((L.box_oct[b] >> a) & 1) ? 0.5 * L.H : -0.5 * L.H;
                for (int32_t sl = Lp->slot_start[p]; sl < Lp->slot_start[p + 1]; ++sl) {
                    int32_t pc = Lp->slot_cone[sl];
                    int pcell = pc / Lp->ns, pis = pc % Lp->ns;
                    for (int a = 0; a < ps; ++a) {
                        double rr = Lp->node_r[(size_t)pis * ps + a];
                        for (int bb = 0; bb < pang; ++bb)
                            for (int cc = 0; cc < pang; ++cc) {
                                const double* dir = &Lp->node_dir[(((size_t)pcell * pang + bb) * pang + cc) * 3];
                                double v[3];
                                node_minus(rr, dir, o, v);
                                ConeLoc cl;
                                cone_locate(v[0], v[1], v[2], L.h, L.ds, L.dang, L.ns, L.nc, cl);
                                mark(b, cl);
                            }
                    }
                }
            }
        }, 1);
        // Compact into per-cell masks and slots.
        if (dilate) {
            std::atomic<int64_t> nd{0};
            parallel_for(L.nbox, [&](int64_t b) {
                int64_t c = 0;
                for (int64_t w = 0; w < wpb; ++w) {
                    uint64_t extra = dil[(size_t)b * wpb + w] & ~prim[(size_t)b * wpb + w];
                    c += __builtin_popcountll(extra);
                    prim[(size_t)b * wpb + w] |= extra;
                }
                nd += c;
            }, 16);
            n_dilated += nd.load();
        }
        std::vector<int32_t> cnt(L.nbox);
        parallel_for(L.nbox, [&](int64_t b) {
            int64_t c = 0;
            for (int64_t w = 0; w < wpb; ++w) c += __builtin_popcountll(prim[(size_t)b * wpb + w]);
            cnt[b] = (int32_t)c;
        }, 16);
        L.slot_start.assign(L.nbox + 1, 0);
        for (int64_t b = 0; b < L.nbox; ++b) {
            if ((int64_t)L.slot_start[b] + cnt[b] > INT32_MAX) {
                code = IFGF_E_UNSUPPORTED;
                return "too many relevant cones at level " + std::to_string(d);
            }
            L.slot_start[b + 1] = L.slot_start[b] + cnt[b];
        }
        L.nslots = L.slot_start[L.nbox];
        reserve_mapped(L.slot_box, L.nslots);
        L.slot_box.resize(L.nslots);
        reserve_mapped(L.slot_cone, L.nslots);
        L.slot_cone.resize(L.nslots);
        reserve_mapped(L.cell_base, (size_t)L.nbox * L.ncell);
        L.cell_base.assign((size_t)L.nbox * L.ncell, 0);
        reserve_mapped(L.cell_mask, (size_t)L.nbox * L.ncell * L.W);
        L.cell_mask.assign((size_t)L.nbox * L.ncell * L.W, 0);
        parallel_for(L.nbox, [&](int64_t b) {
            const uint64_t* P = &prim[(size_t)b * wpb];
            int32_t slot = L.slot_start[b];
            for (int cell = 0; cell < L.ncell; ++cell) {
                L.cell_base[(size_t)b * L.ncell + cell] = slot;
                uint64_t* M = &L.cell_mask[((size_t)b * L.ncell + cell) * L.W];
                int64_t base = (int64_t)cell * L.ns;
                for (int is = 0; is < L.ns; ++is) {
                    int64_t bit = base + is;
                    if ((P[bit >> 6] >> (bit & 63)) & 1ull) {
                        M[is >> 6] |= 1ull << (is & 63);
                        L.slot_box[slot] = (int32_t)b;
                        L.slot_cone[slot] = (int32_t)(base + is);
                        ++slot;
                    }
                }
            }
        }, 1);
        phase(d >= 4 ? "  relevant cones (level)" : "  relevant cones (level 3)");
    }
    for (int d = 1; d < 3 && d <= D; ++d) {
        HostLevel& L = hp.L[d];
        L.slot_start.assign(L.nbox + 1, 0);
    }
    // adaptive octree: the slots of the leaf boxes above level D, and the
    // direct evaluations of every level-D box: the points of each leaf q (on
    // its own level d) that neighbours the box's level-d ancestor
    if (hp.adaptive) {
        for (int d = 3; d < D; ++d) {
            HostLevel& L = hp.L[d];
            for (int64_t b = 0; b < L.nbox; ++b)
                if (L.leaf[b])
                    for (int32_t sl = L.slot_start[b]; sl < L.slot_start[b + 1]; ++sl) L.leaf_slots.push_back(sl);
        }
        const HostLevel& LD = hp.L[D];
        std::vector<std::vector<int32_t>> rng(LD.nbox);
        parallel_for(LD.nbox, [&](int64_t T) {
            int32_t a = (int32_t)T;
            std::vector<int32_t> anc(D + 1, -1);
            for (int d = D; d >= 2; --d) {
                anc[d] = a;
                a = hp.L[d].parent[a];
            }
            for (int d = 2; d <= D; ++d) {
                const HostLevel& L = hp.L[d];
                for (int32_t qi = L.nbr_start[anc[d]]; qi < L.nbr_start[anc[d] + 1]; ++qi) {
                    const int32_t q = L.nbr[qi];
                    if (!L.leaf[q]) continue;
                    rng[T].push_back(L.box_start[q]);
                    rng[T].push_back(L.box_start[q + 1]);
                }
            }
        }, 256);
        hp.near_start.assign(LD.nbox + 1, 0);
        for (int64_t T = 0; T < LD.nbox; ++T) {
            if ((int64_t)hp.near_start[T] + (int64_t)rng[T].size() / 2 > INT32_MAX) {
                code = IFGF_E_UNSUPPORTED;
                return "too many direct-evaluation ranges";
            }
            hp.near_start[T + 1] = hp.near_start[T] + (int32_t)(rng[T].size() / 2);
        }
        hp.near_lo.resize(hp.near_start[LD.nbox]);
        hp.near_hi.resize(hp.near_start[LD.nbox]);
        for (int64_t T = 0; T < LD.nbox; ++T)
            for (size_t e = 0; e < rng[T].size() / 2; ++e) {
                hp.near_lo[hp.near_start[T] + e] = rng[T][2 * e];
                hp.near_hi[hp.near_start[T] + e] = rng[T][2 * e + 1];
            }
    }
    for (int d = 4; d <= D; ++d)
        if (hp.L[d].use_frames && hp.L[d].frame_groups_ok && hp.L[d].ntiles > 0) build_tile_entries(hp, d);
    phase("box tile entries");

    phase("relevant cones, frames, tiles");
    // Cousin-target pair tables, coarse levels first, while the budget lasts.
    {
        const double per = tab_elem_bytes;
        double used = 0.0;
        for (int d = 3; d <= D && per > 0.0; ++d) {
            HostLevel& L = hp.L[d];
            double npairs = 0.0;
            for (int64_t T = 0; T < L.nbox; ++T)
                npairs += (double)(L.box_start[T + 1] - L.box_start[T]) * (L.cou_start[T + 1] - L.cou_start[T]);
            // the table with its cone-ordered copy (two-phase evaluation) if
            // both fit, else the table alone, else no further levels
            const bool both = ord_elem_bytes > 0.0 && used + npairs * (per + ord_elem_bytes) <= pair_budget;
            if (!both && used + npairs * per > pair_budget) break;
            used += npairs * (both ? per + ord_elem_bytes : per);
            if (pairs_device) {
                pair_offsets(L);
                L.use_pairs = true;
                L.pairs_device = true;
                L.pairs_ordered = both;
                continue;
            }
            build_pairs(hp, d);
            if (both) build_pair_order(L);
        }
    }

    phase("cousin-target pair tables");
    // Statistics.
    ifgf_stats& st = hp.stats;
    std::memset(&st, 0, sizeof(st));
    st.D = D;
    st.n_points = (int32_t)n;
    st.H1 = H1;
    for (int a = 0; a < 3; ++a) st.x1[a] = hp.x1[a];
    st.kappa = kappa;
    st.ps = ps;
    st.pang = pang;
    for (int d = 1; d <= D; ++d) {
        const HostLevel& L = hp.L[d];
        st.ns[d] = L.ns;
        st.nc[d] = L.nc;
        st.n_boxes[d] = L.nbox;
        st.n_cones[d] = L.nslots;
        // cousins of the source boxes and the targets in them
        const std::vector<int32_t>& mst = hp.adaptive ? L.mcou_start : L.cou_start;
        const std::vector<int32_t>& mco = hp.adaptive ? L.mcou : L.cou;
        int64_t mx = 0, ce = 0, pe = 0, nc = 0;
        for (int64_t b = 0; b < L.nbox; ++b) {
            st.n_src_boxes[d] += L.active[b];
            st.n_leaf_boxes[d] += L.leaf[b];
            if (!L.active[b] || mst.empty()) continue;
            nc += mst[b + 1] - mst[b];
            mx = std::max<int64_t>(mx, mst[b + 1] - mst[b]);
            for (int32_t ci = mst[b]; ci < mst[b + 1]; ++ci) {
                int32_t c = mco[ci];
                ce += L.box_start[c + 1] - L.box_start[c];
            }
            if (d >= 4) {
                int32_t p = L.parent[b];
                pe += (int64_t)(hp.L[d - 1].slot_start[p + 1] - hp.L[d - 1].slot_start[p]) * hp.P;
            }
        }
        st.n_cousin_boxes[d] = nc;
        st.max_cousin_boxes[d] = mx;
        st.n_cousin_evals[d] = ce;
        st.n_parent_evals[d] = pe;
        st.n_frames[d] = L.nframes;
        st.pairs_tabulated[d] = L.use_pairs ? 1 : 0;
    }
    {
        int64_t leaf = 0, nearp = 0;
        for (int d = 3; d <= D; ++d) {
            const HostLevel& L = hp.L[d];
            for (int64_t b = 0; b < L.nbox; ++b)
                if (L.leaf[b])
                    leaf += (int64_t)(L.slot_start[b + 1] - L.slot_start[b]) * hp.P * (L.box_start[b + 1] - L.box_start[b]);
        }
        const HostLevel& L = hp.L[D];
        for (int64_t b = 0; b < L.nbox; ++b) {
            int64_t nb = L.box_start[b + 1] - L.box_start[b];
            if (hp.adaptive) {
                for (int32_t e = hp.near_start[b]; e < hp.near_start[b + 1]; ++e) nearp += nb * (hp.near_hi[e] - hp.near_lo[e]);
                continue;
            }
            for (int32_t qi = L.nbr_start[b]; qi < L.nbr_start[b + 1]; ++qi) {
                int32_t q = L.nbr[qi];
                nearp += nb * (L.box_start[q + 1] - L.box_start[q]);
            }
        }
        st.n_leaf_pairs = leaf;
        st.n_near_pairs = nearp - n;
    }
    st.n_dilated = n_dilated;
    phase("statistics");
    st.t_plan_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    code = IFGF_OK;
    return std::string();
}

}  // namespace ifgf
