// Plan construction on the GPU (Sec. 3.3.2): the relevant cone segments of
// every level (eq. defallrelevantconesegments) and the cousin-target pair
// tables.  The host builds the box tree (Morton order, relevant boxes,
// neighbours, cousins) and the child-to-parent frames; for each level the
// device
//   1. marks, in one bit per (box, cone), the cone of every cousin point
//      (rule (i)) and the cone of every interpolation point of the parent's
//      relevant cones seen from the child (rule (ii)), with the same
//      cone-coordinate map and face dilation as the host builder;
//   2. numbers the marked cones box by box, cell by cell, radial interval by
//      radial interval -- the host builder's slot order -- from an exclusive
//      scan of the per-word bit counts, and fills the per-cell slot bases and
//      radial masks that the kernels look cones up in;
// and the host takes the slot tables back for the frames, tiles and
// statistics of the next steps.  The pair tables (slot, local coordinates and
// centred factor of every (target, cousin box) pair, and their copy in cone
// order for the two-phase cousin evaluation) are computed directly in device
// memory.
#include <hipcub/hipcub.hpp>

#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "host_mem.hpp"
#include "ifgf_internal.hpp"

namespace ifgf {
namespace {

constexpr int kPB = 256;   // threads per block of the builder kernels

// Blocks of a launch over n items: the builder kernels loop with a stride of
// the whole grid, and the grid stays far below 2^32 work-items (a dispatch
// counts its work-items in 32 bits; rule (ii) alone can pass 4e9 items).
inline unsigned blocks_for(int64_t n)
{
    const int64_t b = (n + kPB - 1) / kPB;
    return (unsigned)(b < ((int64_t)1 << 20) ? (b > 0 ? b : 1) : ((int64_t)1 << 20));
}

#define GRID_LOOP(i, n) for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kPB)

struct Marks {
    unsigned long long* prim;  // [nbox][wpb] cones marked by rules (i) and (ii)
    unsigned long long* dil;   // [nbox][wpb] neighbours of face points (dilation)
    int64_t wpb;               // 64-bit words per box
    int ns, nc;
    double h, ds, dang;
};

// Marks only ever set bits, so a bit seen set is set for good: most marks
// repeat one (every interpolation point of a box's parent cones falls into a
// few of its cones) and end with that load, instead of queueing atomics on
// the few words of one box.
__device__ inline void set_bit(unsigned long long* w, int64_t bit)
{
    unsigned long long* a = w + (bit >> 6);
    const unsigned long long m = 1ull << (bit & 63);
    if (!(__hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & m)) atomicOr(a, m);
}

// The cone of a query point, and with dilation the cones on the other side
// of every face the point lies within kDilateTol of (in local coordinates),
// so that a last-bit difference in the evaluation of the point's cone still
// finds computed data.
__device__ inline void mark_cone(const Marks& M, int64_t b, const ConeLoc& c, int dilate)
{
    unsigned long long* P = M.prim + b * M.wpb;
    set_bit(P, (int64_t)c.cell * M.ns + c.is);
    if (!dilate) return;
    const double tol = kDilateTol;
    int ls[3] = {c.is, c.is, c.is}, lt[3] = {c.it, c.it, c.it}, lp[3] = {c.ip, c.ip, c.ip};
    int nsv = 1, ntv = 1, npv = 1;
    if (c.ts > 1.0 - tol && c.is + 1 < M.ns) ls[nsv++] = c.is + 1;
    if (c.ts < -1.0 + tol && c.is > 0) ls[nsv++] = c.is - 1;
    if (c.tt > 1.0 - tol && c.it + 1 < M.nc) lt[ntv++] = c.it + 1;
    if (c.tt < -1.0 + tol && c.it > 0) lt[ntv++] = c.it - 1;
    if (c.tp > 1.0 - tol) lp[npv++] = (c.ip + 1) % (2 * M.nc);
    if (c.tp < -1.0 + tol) lp[npv++] = (c.ip + 2 * M.nc - 1) % (2 * M.nc);
    if (nsv * ntv * npv == 1) return;
    unsigned long long* Q = M.dil + b * M.wpb;
    for (int i = 0; i < nsv; ++i)
        for (int j = 0; j < ntv; ++j)
            for (int k = 0; k < npv; ++k) set_bit(Q, ((int64_t)lt[j] * 2 * M.nc + lp[k]) * M.ns + ls[i]);
}

// Largest b in [0, n) with start[b] <= x (start ascending, start[0] <= x).
template <typename I>
__device__ inline int owner(const I* start, int n, int64_t x)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)start[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Rule (i): one thread per (box, cousin) entry marks the cones of the
// cousin's points seen from the box.
__global__ void __launch_bounds__(kPB) k_mark_cousin_points(Marks M, int nbox, int64_t ncou,
                                                            const int32_t* __restrict__ cou_start,
                                                            const int32_t* __restrict__ cou,
                                                            const int32_t* __restrict__ box_start,
                                                            const double* __restrict__ box_ctr,
                                                            const double* __restrict__ pts, int dilate)
{
    GRID_LOOP(ci, ncou) {
        const int b = owner(cou_start, nbox, ci);
        const int c = cou[ci];
        const double c0 = box_ctr[3 * b], c1 = box_ctr[3 * b + 1], c2 = box_ctr[3 * b + 2];
        for (int j = box_start[c]; j < box_start[c + 1]; ++j) {
            ConeLoc cl;
            cone_locate(pts[3 * j] - c0, pts[3 * j + 1] - c1, pts[3 * j + 2] - c2, M.h, M.ds, M.dang, M.ns, M.nc, cl);
            mark_cone(M, b, cl, dilate);
        }
    }
}

// Rule (ii): one thread per (child box, parent slot, interpolation point):
// through the frame's tabulated child cone where the level has frames (no
// dilation: the kernels read the same tabulated cone), else the point's
// cone computed in the child's frame.
struct ParentNodes {
    int nbox, P, ps, pang, pns, use_frames;
    double H;                          // child box side
    const int64_t* off;                // [nbox + 1] first (box, parent slot) pair of each child box
    const int32_t* parent;             // [nbox]
    const uint8_t* box_oct;            // [nbox]
    const int32_t* pslot_start;        // parent level [nbox_p + 1]
    const int32_t* pslot_cone;         // parent level [nslots_p]
    const double* pnode_r;             // parent level [pns][ps]
    const double* pnode_dir;           // parent level [ncell_p][pang][pang][3]
    const int32_t* pframe;             // [nslots_p][8] (frames)
    const uint32_t* fr_key;            // [nframes][P] (frames)
};

__global__ void __launch_bounds__(kPB) k_mark_parent_nodes(Marks M, ParentNodes N, int64_t total, int dilate)
{
    GRID_LOOP(gid, total) {
        const int64_t pr = gid / N.P;
        const int nu = (int)(gid - pr * N.P);
        const int b = owner(N.off, N.nbox, pr);
        const int oct = N.box_oct[b];
        const int sl = N.pslot_start[N.parent[b]] + (int)(pr - N.off[b]);
        if (N.use_frames) {
            const int f = N.pframe[(int64_t)sl * 8 + oct];
            set_bit(M.prim + (int64_t)b * M.wpb, N.fr_key[(int64_t)f * N.P + nu]);
            continue;
        }
        const int pc = N.pslot_cone[sl];
        const int pcell = pc / N.pns, pis = pc - pcell * N.pns;
        const int a = nu / (N.pang * N.pang), bc = nu - a * N.pang * N.pang;
        const double rr = N.pnode_r[pis * N.ps + a];
        const double* dir = &N.pnode_dir[((int64_t)pcell * N.pang * N.pang + bc) * 3];
        double o[3];
        for (int x = 0; x < 3; ++x) o[x] = ((oct >> x) & 1) ? 0.5 * N.H : -0.5 * N.H;
        double v[3];
        node_minus(rr, dir, o, v);
        ConeLoc cl;
        cone_locate(v[0], v[1], v[2], M.h, M.ds, M.dang, M.ns, M.nc, cl);
        mark_cone(M, b, cl, dilate);
    }
}

// Folds the dilation marks into the primary ones (counting the cones they
// add) and counts the marked cones of every word.
__global__ void __launch_bounds__(kPB) k_merge_count(unsigned long long* __restrict__ prim,
                                                     const unsigned long long* __restrict__ dil, int64_t nwords,
                                                     int dilate, int64_t* __restrict__ cnt,
                                                     unsigned long long* __restrict__ ndil)
{
    GRID_LOOP(w, nwords) {
        unsigned long long m = prim[w];
        if (dilate) {
            const unsigned long long extra = dil[w] & ~m;
            if (extra) {
                atomicAdd(ndil, (unsigned long long)__popcll(extra));
                m |= extra;
                prim[w] = m;
            }
        }
        cnt[w] = __popcll(m);
    }
}

// Slot tables of the marked cones: slot = number of marked cones before it
// in (box, cell, radial interval) order, from the exclusive scan `woff` of
// the word counts.  One thread per (box, cell).
__global__ void __launch_bounds__(kPB) k_fill_cells(const unsigned long long* __restrict__ prim,
                                                    const int64_t* __restrict__ woff, int64_t wpb, int nbox,
                                                    int ncell, int ns, int W, int32_t* __restrict__ cell_base,
                                                    unsigned long long* __restrict__ cell_mask,
                                                    int32_t* __restrict__ slot_box, int32_t* __restrict__ slot_cone)
{
    GRID_LOOP(gid, (int64_t)nbox * ncell) {
        const int b = (int)(gid / ncell);
        const int cell = (int)(gid - (int64_t)b * ncell);
        const unsigned long long* P = prim + (int64_t)b * wpb;
        const int64_t bit0 = (int64_t)cell * ns;
        const int64_t w0 = bit0 >> 6;
        const unsigned long long below = (bit0 & 63) ? P[w0] & ((1ull << (bit0 & 63)) - 1ull) : 0ull;
        int64_t slot = woff[(int64_t)b * wpb + w0] + __popcll(below);
        cell_base[gid] = (int32_t)slot;
        for (int w = 0; w < W; ++w) {
            unsigned long long m = 0;
            const int i1 = ns < 64 * (w + 1) ? ns : 64 * (w + 1);
            for (int is = 64 * w; is < i1; ++is) {
                const int64_t bit = bit0 + is;
                if ((P[bit >> 6] >> (bit & 63)) & 1ull) {
                    m |= 1ull << (is & 63);
                    slot_box[slot] = b;
                    slot_cone[slot] = (int32_t)bit;
                    ++slot;
                }
            }
            cell_mask[gid * W + w] = m;
        }
    }
}

__global__ void __launch_bounds__(kPB) k_slot_start(const int64_t* __restrict__ woff, int64_t wpb, int nbox,
                                                    int64_t nslots, int32_t* __restrict__ slot_start)
{
    GRID_LOOP(b, (nbox) + 1) {
        slot_start[b] = (int32_t)(b < nbox ? woff[b * wpb] : nslots);
    }
}

// --------------------------------------------------- device buffer helpers

class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void reset()
    {
        if (p_) (void)hipFree(p_);
        p_ = nullptr;
        n_ = 0;
    }
    hipError_t alloc(size_t bytes)
    {
        if (bytes <= n_ && p_) return hipSuccess;
        reset();
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&p_, bytes);
        if (e == hipSuccess) n_ = bytes;
        return e;
    }
    template <typename T>
    hipError_t put(const std::vector<T>& v)
    {
        hipError_t e = alloc(v.size() * sizeof(T));
        if (e != hipSuccess || v.empty()) return e;
        return hipMemcpy(p_, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    }
    template <typename T>
    T* as() const { return (T*)p_; }

  private:
    void* p_ = nullptr;
    size_t n_ = 0;
};

template <typename T>
hipError_t get(std::vector<T>& v, const DevBuf& b, size_t n)
{
    reserve_mapped(v, n);
    v.resize(n);
    if (n == 0) return hipSuccess;
    return hipMemcpy(v.data(), b.as<T>(), n * sizeof(T), hipMemcpyDeviceToHost);
}

#define IFGF_TRY(x)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess) {                                                                      \
            code = IFGF_E_HIP;                                                                       \
            return std::string("device plan: ") + #x + ": " + hipGetErrorString(e_);                 \
        }                                                                                            \
    } while (0)

class GpuConeMarker : public ConeMarker {
  public:
    std::string mark_level(HostPlan& hp, int d, bool dilate, int64_t& n_dilated, ifgf_status& code) override
    {
        HostLevel& L = hp.L[d];
        if (!pts_ready_) {
            IFGF_TRY(pts_.put(hp.pts));
            pts_ready_ = true;
        }
        const int64_t ncone = (int64_t)L.ncell * L.ns;
        const int64_t wpb = (ncone + 63) / 64;
        const int64_t nwords = L.nbox * wpb;
        IFGF_TRY(prim_.alloc(nwords * 8));
        IFGF_TRY(hipMemset(prim_.as<void>(), 0, nwords * 8));
        if (dilate) {
            IFGF_TRY(dil_.alloc(nwords * 8));
            IFGF_TRY(hipMemset(dil_.as<void>(), 0, nwords * 8));
        }
        Marks M{prim_.as<unsigned long long>(), dil_.as<unsigned long long>(), wpb, L.ns, L.nc, L.h, L.ds, L.dang};
        // rule (i)
        IFGF_TRY(box_start_.put(L.box_start));
        IFGF_TRY(box_ctr_.put(L.box_ctr));
        // every cousin of the source boxes (adaptive octree: cou holds only
        // the cousins that are source boxes themselves)
        const std::vector<int32_t>& mst = hp.adaptive ? L.mcou_start : L.cou_start;
        IFGF_TRY(cou_start_.put(mst));
        IFGF_TRY(cou_.put(hp.adaptive ? L.mcou : L.cou));
        const int64_t ncou = mst[L.nbox];
        if (ncou > 0)
            k_mark_cousin_points<<<blocks_for(ncou), kPB>>>(M, (int)L.nbox, ncou, cou_start_.as<int32_t>(),
                                                            cou_.as<int32_t>(), box_start_.as<int32_t>(),
                                                            box_ctr_.as<double>(), pts_.as<double>(), dilate ? 1 : 0);
        IFGF_TRY(hipGetLastError());
        // rule (ii)
        if (d >= 4) {
            const HostLevel& Lp = hp.L[d - 1];
            std::vector<int64_t> off(L.nbox + 1, 0);
            for (int64_t b = 0; b < L.nbox; ++b) {
                const int32_t p = L.parent[b];
                off[b + 1] = off[b] + (L.active[b] ? Lp.slot_start[p + 1] - Lp.slot_start[p] : 0);
            }
            const int64_t total = off[L.nbox] * hp.P;
            IFGF_TRY(off_.put(off));
            IFGF_TRY(parent_.put(L.parent));
            IFGF_TRY(box_oct_.put(L.box_oct));
            IFGF_TRY(pnode_r_.put(Lp.node_r));
            IFGF_TRY(pnode_dir_.put(Lp.node_dir));
            if (L.use_frames) {
                IFGF_TRY(pframe_.put(L.pframe));
                IFGF_TRY(fr_key_.put(L.fr_key));
            }
            ParentNodes N{(int)L.nbox, hp.P, hp.ps, hp.pang, Lp.ns, L.use_frames ? 1 : 0, L.H,
                          off_.as<int64_t>(), parent_.as<int32_t>(), box_oct_.as<uint8_t>(),
                          pslot_start_.as<int32_t>(), pslot_cone_.as<int32_t>(), pnode_r_.as<double>(),
                          pnode_dir_.as<double>(), pframe_.as<int32_t>(), fr_key_.as<uint32_t>()};
            if (total > 0) k_mark_parent_nodes<<<blocks_for(total), kPB>>>(M, N, total, dilate ? 1 : 0);
            IFGF_TRY(hipGetLastError());
            if (L.use_frames) {
                pframe_.reset();
                fr_key_.reset();
            }
        }
        // numbering
        IFGF_TRY(cnt_.alloc(nwords * 8));
        IFGF_TRY(woff_.alloc(nwords * 8));
        IFGF_TRY(ndil_.alloc(8));
        IFGF_TRY(hipMemset(ndil_.as<void>(), 0, 8));
        k_merge_count<<<blocks_for(nwords), kPB>>>(prim_.as<unsigned long long>(), dil_.as<unsigned long long>(),
                                                   nwords, dilate ? 1 : 0, cnt_.as<int64_t>(),
                                                   ndil_.as<unsigned long long>());
        IFGF_TRY(hipGetLastError());
        size_t tb = 0;
        IFGF_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt_.as<int64_t>(), woff_.as<int64_t>(), nwords));
        IFGF_TRY(tmp_.alloc(tb));
        IFGF_TRY(hipcub::DeviceScan::ExclusiveSum(tmp_.as<void>(), tb, cnt_.as<int64_t>(), woff_.as<int64_t>(),
                                                  nwords));
        int64_t last[2] = {0, 0};
        IFGF_TRY(hipMemcpy(&last[0], woff_.as<int64_t>() + (nwords - 1), 8, hipMemcpyDeviceToHost));
        IFGF_TRY(hipMemcpy(&last[1], cnt_.as<int64_t>() + (nwords - 1), 8, hipMemcpyDeviceToHost));
        const int64_t nslots = last[0] + last[1];
        unsigned long long nd = 0;
        IFGF_TRY(hipMemcpy(&nd, ndil_.as<void>(), 8, hipMemcpyDeviceToHost));
        n_dilated += (int64_t)nd;
        if (nslots > INT32_MAX) {
            code = IFGF_E_UNSUPPORTED;
            return "too many relevant cones at level " + std::to_string(d);
        }
        const int64_t ncells = L.nbox * L.ncell;
        IFGF_TRY(pslot_start_.alloc((L.nbox + 1) * 4));
        IFGF_TRY(pslot_cone_.alloc(nslots * 4));
        IFGF_TRY(slot_box_.alloc(nslots * 4));
        IFGF_TRY(cell_base_.alloc(ncells * 4));
        IFGF_TRY(cell_mask_.alloc(ncells * L.W * 8));
        k_fill_cells<<<blocks_for(ncells), kPB>>>(prim_.as<unsigned long long>(), woff_.as<int64_t>(), wpb,
                                                  (int)L.nbox, L.ncell, L.ns, L.W, cell_base_.as<int32_t>(),
                                                  cell_mask_.as<unsigned long long>(), slot_box_.as<int32_t>(),
                                                  pslot_cone_.as<int32_t>());
        IFGF_TRY(hipGetLastError());
        k_slot_start<<<blocks_for(L.nbox + 1), kPB>>>(woff_.as<int64_t>(), wpb, (int)L.nbox, nslots,
                                                      pslot_start_.as<int32_t>());
        IFGF_TRY(hipGetLastError());
        // the host takes the tables; the slot starts and cones stay on the
        // device for the next level's rule (ii)
        L.nslots = nslots;
        IFGF_TRY(get(L.slot_start, pslot_start_, (size_t)L.nbox + 1));
        IFGF_TRY(get(L.slot_cone, pslot_cone_, (size_t)nslots));
        IFGF_TRY(get(L.slot_box, slot_box_, (size_t)nslots));
        IFGF_TRY(get(L.cell_base, cell_base_, (size_t)ncells));
        IFGF_TRY(get(L.cell_mask, cell_mask_, (size_t)(ncells * L.W)));
        return std::string();
    }

  private:
    bool pts_ready_ = false;
    DevBuf pts_, prim_, dil_, box_start_, box_ctr_, cou_start_, cou_, off_, parent_, box_oct_, pnode_r_, pnode_dir_,
        pframe_, fr_key_, cnt_, woff_, ndil_, tmp_, pslot_start_, pslot_cone_, slot_box_, cell_base_, cell_mask_;
};

#undef IFGF_TRY

// ------------------------------------------------------------ pair tables

// One thread per (target box T, cousin c of T, target t of T) pair, at entry
// pair_base[T] + c n_T + t: the slot of the cousin's cone containing the
// target, the target's local coordinates in it and G(x_t, x_c).
template <typename T>
__global__ void __launch_bounds__(kPB) k_pair_table(LevelDev L, const double* __restrict__ pts, double kappa,
                                                    int64_t np, int32_t* __restrict__ pr_slot, T* __restrict__ pr_t,
                                                    T* __restrict__ pr_g)
{
    GRID_LOOP(e, np) {
        const int tb = owner(L.pair_base, L.nbox, e);
        const int nT = L.box_start[tb + 1] - L.box_start[tb];
        const int64_t rel = e - L.pair_base[tb];
        const int cl_i = (int)(rel / nT), t = (int)(rel - (int64_t)cl_i * nT);
        const int c = L.cou[L.cou_start[tb] + cl_i];
        const int j = L.box_start[tb] + t;
        ConeLoc cl;
        cone_locate(pts[3 * j] - L.box_ctr[3 * c], pts[3 * j + 1] - L.box_ctr[3 * c + 1], pts[3 * j + 2] - L.box_ctr[3 * c + 2],
                    L.h, L.ds, L.dang, L.ns, L.nc, cl);
        pr_slot[e] = lookup(L, c, cl.cell, cl.is);
        pr_t[e] = (T)cl.ts;
        pr_t[np + e] = (T)cl.tt;
        pr_t[2 * np + e] = (T)cl.tp;
        double s, co;
        sincos(kappa * cl.r, &s, &co);
        const double inv = 1.0 / (4.0 * kPi) / cl.r;
        pr_g[e] = (T)(co * inv);
        pr_g[np + e] = (T)(s * inv);
    }
}

__global__ void __launch_bounds__(kPB) k_pair_keys(const int32_t* __restrict__ pr_slot, int64_t np,
                                                   uint32_t* __restrict__ key, int32_t* __restrict__ idx,
                                                   int32_t* __restrict__ cnt)
{
    GRID_LOOP(e, np) {
        const int32_t s = pr_slot[e];
        key[e] = s >= 0 ? (uint32_t)s : 0xffffffffu;   // pairs without a cone sort last
        idx[e] = (int32_t)e;
        if (s >= 0) atomicAdd(&cnt[s], 1);
    }
}

__global__ void __launch_bounds__(kPB) k_pad_counts(const int32_t* __restrict__ cnt, int64_t nslots,
                                                    int64_t* __restrict__ ucnt, int64_t* __restrict__ pcnt)
{
    GRID_LOOP(s, nslots) {
        ucnt[s] = cnt[s];
        pcnt[s] = (cnt[s] + kPairQuad - 1) / kPairQuad * kPairQuad;
    }
}

// Entry i of the slot-sorted pairs goes to position start[s] + (i - ustart[s])
// of the cone-ordered copy (runs of one slot keep target order: the sort is
// stable).
template <typename T>
__global__ void __launch_bounds__(kPB) k_pair_scatter(const uint32_t* __restrict__ skey,
                                                      const int32_t* __restrict__ sidx, int64_t nvalid,
                                                      const int64_t* __restrict__ ustart,
                                                      const int64_t* __restrict__ start, int64_t np, int64_t no,
                                                      const T* __restrict__ pr_t, const T* __restrict__ pr_g,
                                                      int32_t* __restrict__ pr_order, int32_t* __restrict__ pro_slot,
                                                      T* __restrict__ pro_t, T* __restrict__ pro_g)
{
    GRID_LOOP(i, nvalid) {
        const int64_t s = skey[i];
        const int64_t pos = start[s] + (i - ustart[s]);
        const int64_t e = sidx[i];
        pr_order[pos] = (int32_t)e;
        pro_slot[pos] = (int32_t)s;
        for (int c = 0; c < 3; ++c) pro_t[c * no + pos] = pr_t[c * np + e];
        for (int c = 0; c < 2; ++c) pro_g[c * no + pos] = pr_g[c * np + e];
    }
}

// Placeholders after each slot's run (place -1, the slot's cone, zero
// coordinates and factor).
template <typename T>
__global__ void __launch_bounds__(kPB) k_pair_padding(const int32_t* __restrict__ cnt,
                                                      const int64_t* __restrict__ start, int64_t nslots, int64_t no,
                                                      int32_t* __restrict__ pr_order, int32_t* __restrict__ pro_slot,
                                                      T* __restrict__ pro_t, T* __restrict__ pro_g)
{
    GRID_LOOP(s, nslots) {
        const int64_t end = s + 1 < nslots ? start[s + 1] : no;
        for (int64_t pos = start[s] + cnt[s]; pos < end; ++pos) {
            pr_order[pos] = -1;
            pro_slot[pos] = (int32_t)s;
            for (int c = 0; c < 3; ++c) pro_t[c * no + pos] = (T)0;
            for (int c = 0; c < 2; ++c) pro_g[c * no + pos] = (T)0;
        }
    }
}

template <typename T>
hipError_t pairs_t(DevicePlan& p, int d, bool ordered)
{
    HostLevel& H = p.hp.L[d];
    LevelDev& L = p.L[d];
    const int64_t np = H.pair_base[H.nbox];
    hipError_t e;
    auto dalloc = [&](size_t bytes, void** out) -> hipError_t {
        if (bytes == 0) bytes = 16;
        hipError_t err = hipMalloc(out, bytes);
        if (err == hipSuccess) {
            p.allocs.push_back(*out);
            p.tree_bytes += bytes;
        }
        return err;
    };
    void* q = nullptr;
    {
        std::vector<long long> pb(H.pair_base.begin(), H.pair_base.end());
        if ((e = dalloc(pb.size() * sizeof(long long), &q)) != hipSuccess) return e;
        if ((e = hipMemcpy(q, pb.data(), pb.size() * sizeof(long long), hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        L.pair_base = (const long long*)q;
    }
    int32_t* pr_slot;
    T *pr_t, *pr_g;
    if ((e = dalloc((size_t)np * 4, &q)) != hipSuccess) return e;
    pr_slot = (int32_t*)q;
    if ((e = dalloc((size_t)np * 3 * sizeof(T), &q)) != hipSuccess) return e;
    pr_t = (T*)q;
    if ((e = dalloc((size_t)np * 2 * sizeof(T), &q)) != hipSuccess) return e;
    pr_g = (T*)q;
    L.npairs_cou = np;
    L.pr_slot = pr_slot;
    L.pr_t = pr_t;
    L.pr_g = pr_g;
    L.npairs_ord = 0;
    if (np > 0) k_pair_table<T><<<blocks_for(np), kPB>>>(L, p.pts, p.hp.kappa, np, pr_slot, pr_t, pr_g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!ordered || np == 0) return hipStreamSynchronize(nullptr);
    // the cone-ordered copy: stable sort of the pairs by slot
    const int64_t ns = H.nslots;
    if (ns == 0) return hipStreamSynchronize(nullptr);
    DevBuf key, idx, skey, sidx, cnt, ucnt, pcnt, ustart, start, tmp;
    if ((e = key.alloc(np * 4)) != hipSuccess || (e = idx.alloc(np * 4)) != hipSuccess ||
        (e = skey.alloc(np * 4)) != hipSuccess || (e = sidx.alloc(np * 4)) != hipSuccess ||
        (e = cnt.alloc(ns * 4)) != hipSuccess || (e = ucnt.alloc(ns * 8)) != hipSuccess ||
        (e = pcnt.alloc(ns * 8)) != hipSuccess || (e = ustart.alloc(ns * 8)) != hipSuccess ||
        (e = start.alloc(ns * 8)) != hipSuccess)
        return e;
    if ((e = hipMemset(cnt.as<void>(), 0, ns * 4)) != hipSuccess) return e;
    k_pair_keys<<<blocks_for(np), kPB>>>(pr_slot, np, key.as<uint32_t>(), idx.as<int32_t>(), cnt.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    size_t tb = 0, tb2 = 0;
    if ((e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key.as<uint32_t>(), skey.as<uint32_t>(), idx.as<int32_t>(),
                                                sidx.as<int32_t>(), (int)np)) != hipSuccess)
        return e;
    if ((e = hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, ucnt.as<int64_t>(), ustart.as<int64_t>(), (int)ns)) !=
        hipSuccess)
        return e;
    if ((e = tmp.alloc(tb > tb2 ? tb : tb2)) != hipSuccess) return e;
    if ((e = hipcub::DeviceRadixSort::SortPairs(tmp.as<void>(), tb, key.as<uint32_t>(), skey.as<uint32_t>(),
                                                idx.as<int32_t>(), sidx.as<int32_t>(), (int)np)) != hipSuccess)
        return e;
    k_pad_counts<<<blocks_for(ns), kPB>>>(cnt.as<int32_t>(), ns, ucnt.as<int64_t>(), pcnt.as<int64_t>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipcub::DeviceScan::ExclusiveSum(tmp.as<void>(), tb2, ucnt.as<int64_t>(), ustart.as<int64_t>(),
                                              (int)ns)) != hipSuccess)
        return e;
    if ((e = hipcub::DeviceScan::ExclusiveSum(tmp.as<void>(), tb2, pcnt.as<int64_t>(), start.as<int64_t>(),
                                              (int)ns)) != hipSuccess)
        return e;
    int64_t tail[4];
    if ((e = hipMemcpy(&tail[0], start.as<int64_t>() + (ns - 1), 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    if ((e = hipMemcpy(&tail[1], pcnt.as<int64_t>() + (ns - 1), 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    if ((e = hipMemcpy(&tail[2], ustart.as<int64_t>() + (ns - 1), 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    if ((e = hipMemcpy(&tail[3], ucnt.as<int64_t>() + (ns - 1), 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    const int64_t no = tail[0] + tail[1], nvalid = tail[2] + tail[3];
    if (no > INT32_MAX) return hipErrorInvalidValue;
    int32_t *pr_order, *pro_slot;
    T *pro_t, *pro_g;
    if ((e = dalloc((size_t)no * 4, &q)) != hipSuccess) return e;
    pr_order = (int32_t*)q;
    if ((e = dalloc((size_t)no * 4, &q)) != hipSuccess) return e;
    pro_slot = (int32_t*)q;
    if ((e = dalloc((size_t)no * 3 * sizeof(T), &q)) != hipSuccess) return e;
    pro_t = (T*)q;
    if ((e = dalloc((size_t)no * 2 * sizeof(T), &q)) != hipSuccess) return e;
    pro_g = (T*)q;
    if (nvalid > 0)
        k_pair_scatter<T><<<blocks_for(nvalid), kPB>>>(skey.as<uint32_t>(), sidx.as<int32_t>(), nvalid,
                                                       ustart.as<int64_t>(), start.as<int64_t>(), np, no, pr_t, pr_g,
                                                       pr_order, pro_slot, pro_t, pro_g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_pair_padding<T><<<blocks_for(ns), kPB>>>(cnt.as<int32_t>(), start.as<int64_t>(), ns, no, pr_order, pro_slot,
                                               pro_t, pro_g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    L.npairs_ord = no;
    L.pr_order = pr_order;
    L.pro_slot = pro_slot;
    L.pro_t = pro_t;
    L.pro_g = pro_g;
    return hipStreamSynchronize(nullptr);
}

// One thread per (target box T, cousin c, target t) pair of a level without
// a pair table, at entry pair_off[T] + c n_T + t: the slot of the cousin's
// cone that holds the target (the sort key; pairs without one sort last and
// are counted) and the pair packed as (target point, c).
__global__ void __launch_bounds__(kPB) k_go_keys(LevelDev L, const double* __restrict__ pts,
                                                 const long long* __restrict__ pair_off, int64_t np,
                                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                 int32_t* __restrict__ cnt, unsigned long long* __restrict__ nmiss)
{
    GRID_LOOP(e, np) {
        const int tb = owner(pair_off, L.nbox, e);
        const int b0 = L.box_start[tb];
        const int nT = L.box_start[tb + 1] - b0;
        const int64_t rel = e - pair_off[tb];
        const int ci = (int)(rel / nT), t = (int)(rel - (int64_t)ci * nT);
        const int c = L.cou[L.cou_start[tb] + ci];
        const int j = b0 + t;
        ConeLoc cl;
        cone_locate(pts[3 * j] - L.box_ctr[3 * c], pts[3 * j + 1] - L.box_ctr[3 * c + 1],
                    pts[3 * j + 2] - L.box_ctr[3 * c + 2], L.h, L.ds, L.dang, L.ns, L.nc, cl);
        const int s = lookup(L, c, cl.cell, cl.is);
        key[e] = s >= 0 ? (uint32_t)s : 0xffffffffu;
        val[e] = (uint32_t)j | ((uint32_t)ci << 24);
        if (s >= 0) atomicAdd(&cnt[s], 1);
        else atomicAdd(nmiss, 1ull);
    }
}

// Entry i of the slot-sorted pairs goes to position start[s] + (i -
// ustart[s]) of the order; the places after each slot's run are padding.
__global__ void __launch_bounds__(kPB) k_go_scatter(const uint32_t* __restrict__ skey,
                                                    const uint32_t* __restrict__ sval, int64_t nvalid,
                                                    const int64_t* __restrict__ ustart,
                                                    const int64_t* __restrict__ start, uint32_t* __restrict__ ord)
{
    GRID_LOOP(i, nvalid) {
        const int64_t s = skey[i];
        ord[start[s] + (i - ustart[s])] = sval[i];
    }
}

__global__ void __launch_bounds__(kPB) k_go_padding(const int32_t* __restrict__ cnt,
                                                    const int64_t* __restrict__ start, int64_t nslots, int64_t no,
                                                    uint32_t* __restrict__ ord)
{
    GRID_LOOP(s, nslots) {
        const int64_t end = s + 1 < nslots ? start[s + 1] : no;
        for (int64_t pos = start[s] + cnt[s]; pos < end; ++pos) ord[pos] = 0xffffffffu;
    }
}

}  // namespace

namespace {

hipError_t pair_order(DevicePlan& p, int d, double budget);

}  // namespace

// The order is an optimisation: where its buffers do not fit the device, the
// level keeps the per-pair evaluation and the plan is built all the same.
hipError_t build_pair_order_device(DevicePlan& p, int d, double budget)
{
    hipError_t e = pair_order(p, d, budget);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        p.go_ord[d] = nullptr;
        p.ngo[d] = 0;
        return hipSuccess;
    }
    return e;
}

namespace {

hipError_t pair_order(DevicePlan& p, int d, double budget)
{
    const HostLevel& H = p.hp.L[d];
    const LevelDev& L = p.L[d];
    const int64_t np = p.npairs_all[d];
    const int64_t ns = H.nslots;
    p.go_ord[d] = nullptr;
    p.ngo[d] = 0;
    if (np <= 0 || np > INT32_MAX || ns <= 0 || !p.pair_off[d] || p.hp.n >= ((int64_t)1 << 24)) return hipSuccess;
    for (int64_t T = 0; T < H.nbox; ++T)
        if (H.cou_start[T + 1] - H.cou_start[T] > 255) return hipSuccess;
    // padded size bound: every slot's run rounded up to kPairQuad
    if ((double)(np + (int64_t)(kPairQuad - 1) * ns) * 4.0 > budget) return hipSuccess;
    hipError_t e;
    DevBuf key, val, skey, sval, cnt, ucnt, pcnt, ustart, start, tmp, miss;
    if ((e = key.alloc(np * 4)) != hipSuccess || (e = val.alloc(np * 4)) != hipSuccess ||
        (e = skey.alloc(np * 4)) != hipSuccess || (e = sval.alloc(np * 4)) != hipSuccess ||
        (e = cnt.alloc(ns * 4)) != hipSuccess || (e = ucnt.alloc(ns * 8)) != hipSuccess ||
        (e = pcnt.alloc(ns * 8)) != hipSuccess || (e = ustart.alloc(ns * 8)) != hipSuccess ||
        (e = start.alloc(ns * 8)) != hipSuccess || (e = miss.alloc(8)) != hipSuccess)
        return e;
    if ((e = hipMemset(cnt.as<void>(), 0, ns * 4)) != hipSuccess) return e;
    if ((e = hipMemset(miss.as<void>(), 0, 8)) != hipSuccess) return e;
    k_go_keys<<<blocks_for(np), kPB>>>(L, p.pts, p.pair_off[d], np, key.as<uint32_t>(), val.as<uint32_t>(),
                                       cnt.as<int32_t>(), miss.as<unsigned long long>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    unsigned long long nmiss = 0;
    if ((e = hipMemcpy(&nmiss, miss.as<void>(), 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    if (nmiss > 0) return hipSuccess;          // keep the per-pair path, which counts the misses
    size_t tb = 0, tb2 = 0;
    if ((e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key.as<uint32_t>(), skey.as<uint32_t>(),
                                                val.as<uint32_t>(), sval.as<uint32_t>(), (int)np)) != hipSuccess)
        return e;
    if ((e = hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, ucnt.as<int64_t>(), ustart.as<int64_t>(), (int)ns)) !=
        hipSuccess)
        return e;
    if ((e = tmp.alloc(tb > tb2 ? tb : tb2)) != hipSuccess) return e;
    if ((e = hipcub::DeviceRadixSort::SortPairs(tmp.as<void>(), tb, key.as<uint32_t>(), skey.as<uint32_t>(),
                                                val.as<uint32_t>(), sval.as<uint32_t>(), (int)np)) != hipSuccess)
        return e;
    key.reset();
    val.reset();
    k_pad_counts<<<blocks_for(ns), kPB>>>(cnt.as<int32_t>(), ns, ucnt.as<int64_t>(), pcnt.as<int64_t>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipcub::DeviceScan::ExclusiveSum(tmp.as<void>(), tb2, ucnt.as<int64_t>(), ustart.as<int64_t>(),
                                              (int)ns)) != hipSuccess)
        return e;
    if ((e = hipcub::DeviceScan::ExclusiveSum(tmp.as<void>(), tb2, pcnt.as<int64_t>(), start.as<int64_t>(),
                                              (int)ns)) != hipSuccess)
        return e;
    int64_t tail[2];
    if ((e = hipMemcpy(&tail[0], start.as<int64_t>() + (ns - 1), 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    if ((e = hipMemcpy(&tail[1], pcnt.as<int64_t>() + (ns - 1), 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    const int64_t no = tail[0] + tail[1];
    void* q = nullptr;
    if ((e = hipMalloc(&q, (size_t)no * 4)) != hipSuccess) return e;
    p.allocs.push_back(q);
    p.tree_bytes += (size_t)no * 4;
    uint32_t* ord = (uint32_t*)q;
    k_go_scatter<<<blocks_for(np), kPB>>>(skey.as<uint32_t>(), sval.as<uint32_t>(), np, ustart.as<int64_t>(),
                                          start.as<int64_t>(), ord);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_go_padding<<<blocks_for(ns), kPB>>>(cnt.as<int32_t>(), start.as<int64_t>(), ns, no, ord);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return e;
    p.go_ord[d] = ord;
    p.ngo[d] = no;
    return hipSuccess;
}

}  // namespace

std::unique_ptr<ConeMarker> make_gpu_cone_marker() { return std::unique_ptr<ConeMarker>(new GpuConeMarker()); }

hipError_t build_pairs_device(DevicePlan& p, int d, bool ordered)
{
    return p.precision == IFGF_MIXED ? pairs_t<float>(p, d, ordered) : pairs_t<double>(p, d, ordered);
}

}  // namespace ifgf
