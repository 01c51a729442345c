// Internal types of the IFGF library: host-built hierarchy, its device
// mirror, and the cone-coordinate map shared by the plan builder (host) and
// the kernels (device).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ifgf.h"

namespace ifgf {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxNodes = 8;       // Chebyshev nodes per direction, upper bound
constexpr int kMaxRhsPass = 16;    // right-hand sides handled by one kernel pass
constexpr double kDilateTol = 1e-9;
constexpr int kMaxFrameGroups = 40;  // distinct child cones one frame may touch
constexpr int kBoxTile = 16;        // parent slots (boxes) of one parent cone per box tile
constexpr int kPairQuad = 4;        // cone-ordered cousin pairs share a cone in runs of this length
// child-to-parent kernel variants (ifgf_plan_autotune, ifgf_plan_kernel_choice)
enum { kC2PGeometry = 0, kC2PFrames = 1, kC2PLds = 2, kC2PMfma = 3, kC2PMfmaGeometry = 4, kC2PBoxes = 5,
       kC2PQuads = 6, kC2PLdsTiled = 7, kC2PBoxAcc = 8, kC2PBoxAccHalf = 9, kC2PVariants = 10 };

// Chebyshev nodes t_k = cos((2k+1) pi / (2n)) on [-1, 1] and the inverse
// denominators of their Lagrange polynomials, 1 / prod_{j != k} (t_k - t_j).
struct ChebNodes {
    double t[kMaxNodes];
    double inv[kMaxNodes];
};

inline ChebNodes make_cheb_nodes(int n)
{
    ChebNodes c{};
    for (int k = 0; k < n; ++k) c.t[k] = std::cos((2.0 * k + 1.0) * kPi / (2.0 * n));
    for (int k = 0; k < n; ++k) {
        double p = 1.0;
        for (int j = 0; j < n; ++j)
            if (j != k) p *= (c.t[k] - c.t[j]);
        c.inv[k] = 1.0 / p;
    }
    return c;
}

// Cone segment of a point: cell = i_theta * (2 n_C) + i_phi, radial index
// i_s, local coordinates (ts, tt, tp) in [-1, 1], and r = |v|.
struct ConeLoc {
    int cell, is, it, ip;
    double ts, tt, tp;
    double r, s, th, ph;
};

// Cone-coordinate map of v = x - x_k (Sec. 3.1-3.2): s = h / |v| with h the
// box circumradius, theta = atan2(sqrt(vx^2 + vy^2), vz) in [0, pi],
// phi = atan2(vy, vx) moved into [0, 2 pi).  The cone intervals are
// half-open (eq. defconedomain), so a point on a face belongs to the interval
// above it: with q = coordinate / interval length the index is
// floor(q + 1e-10), which also keeps points that lie exactly on a face (for
// instance on the planes x = +-y of a symmetric point set) from moving between
// cones with last-bit differences of atan2; phi wraps at 2 pi, s and theta are
// clamped to their last interval.  Contraction into FMAs is switched off so
// that the host (plan) and the device (kernels) form every intermediate with
// the same roundings.
__host__ __device__ inline void cone_locate(double vx, double vy, double vz, double h, double ds,
                                            double dang, int ns, int nc, ConeLoc& c)
{
#pragma clang fp contract(off)
    const double tie = 1e-10;
    double rho2 = vx * vx + vy * vy;
    double r = sqrt(rho2 + vz * vz);
    double s = h / r;
    double th = atan2(sqrt(rho2), vz);
    double ph = atan2(vy, vx);
    if (ph < 0.0) ph += 2.0 * kPi;
    double qs = s / ds, qt = th / dang, qp = ph / dang;
    int is = (int)floor(qs + tie);
    int it = (int)floor(qt + tie);
    int ip = (int)floor(qp + tie);
    if (ip >= 2 * nc) {
        ip -= 2 * nc;
        qp -= 2 * nc;
    }
    is = is < 0 ? 0 : (is > ns - 1 ? ns - 1 : is);
    it = it < 0 ? 0 : (it > nc - 1 ? nc - 1 : it);
    ip = ip < 0 ? 0 : (ip > 2 * nc - 1 ? 2 * nc - 1 : ip);
    c.is = is;
    c.it = it;
    c.ip = ip;
    c.cell = it * (2 * nc) + ip;
    c.ts = 2.0 * (qs - is) - 1.0;
    c.tt = 2.0 * (qt - it) - 1.0;
    c.tp = 2.0 * (qp - ip) - 1.0;
    c.r = r;
    c.s = s;
    c.th = th;
    c.ph = ph;
}

// Position of an interpolation point relative to a child box centre:
// v = r * dir - o, where r * dir is the point relative to the parent centre
// and o the child centre relative to the parent centre.  Formed without
// contraction so that host and device agree bit for bit.
__host__ __device__ inline void node_minus(double rr, const double* dir, const double* o, double* v)
{
#pragma clang fp contract(off)
    v[0] = rr * dir[0] - o[0];
    v[1] = rr * dir[1] - o[1];
    v[2] = rr * dir[2] - o[2];
}

// ------------------------------------------------------------ host plan

struct HostLevel {
    double H = 0, h = 0, ds = 0, dang = 0;
    int ns = 0, nc = 0, ncell = 0, W = 0;     // W: 64-bit mask words per cell
    int64_t nbox = 0;
    std::vector<uint64_t> prefix;             // Morton prefix of each box (sorted)
    std::vector<int32_t> box_start;           // [nbox+1] Morton point ranges
    std::vector<double> box_ctr;              // [nbox][3]
    std::vector<uint8_t> box_oct;             // [nbox] parity bits of the index
    std::vector<int32_t> pt_box;              // [n] box of each Morton point
    std::vector<int32_t> parent;              // [nbox] index at level d-1
    std::vector<int32_t> chl_start, chl;      // children (level d+1)
    std::vector<int32_t> nbr_start, nbr;      // neighbours incl. self
    std::vector<int32_t> cou_start, cou;      // cousins that are source boxes (all of
                                              // them unless the tree is adaptive)
    // adaptive octree: the source tree (active boxes) and its leaves; the
    // cousins of every active box, source boxes or not, for relevance rule
    // (i) (empty when the tree is not adaptive: cou serves)
    std::vector<uint8_t> active, leaf;        // [nbox]
    std::vector<int32_t> mcou_start, mcou;
    std::vector<int32_t> leaf_slots;          // slots of the leaf boxes (levels 3..D-1)
    // relevant cones
    std::vector<int32_t> cell_base;           // [nbox][ncell] first slot
    std::vector<uint64_t> cell_mask;          // [nbox][ncell][W]
    std::vector<int32_t> slot_start;          // [nbox+1]
    std::vector<int32_t> slot_box;            // [nslots]
    std::vector<int32_t> slot_cone;           // [nslots] cell * ns + is
    int64_t nslots = 0;
    std::vector<double> node_r;               // [ns][PS] h / s at radial nodes
    std::vector<double> node_dir;             // [ncell][PA][PA][3] unit directions
    // Child-to-parent frames (levels d >= 4, children at d).  The geometry of
    // the interpolation points of a parent cone gamma seen from the child in
    // octant o depends on (gamma, o) only, not on the boxes; a "frame" holds it
    // for the P points: child cone key (cell * ns + is), local coordinates in
    // the child cone, and the re-centring ratio G(x, x_k) / G(x, x_j).
    std::vector<int32_t> child_of;            // [nbox_{d-1}][8] child in octant o, -1
    bool use_frames = false;                  // frames are shared enough to pay
    int64_t npairs = 0;                       // (parent slot, child) pairs
    int64_t nframes = 0;
    std::vector<int32_t> pframe;              // [nslots_{d-1}][8] frame id, -1: no child
    std::vector<uint32_t> fr_key;             // [nframes][P]
    std::vector<double> fr_t;                 // [nframes][P][3]
    std::vector<double> fr_ratio;             // [nframes][P][2]
    // the distinct child cones of each frame ("groups") and the group of
    // every interpolation point, for staging child cones in LDS
    bool frame_groups_ok = false;             // every frame has <= kMaxFrameGroups
    int fr_max_groups = 0;                    // the most groups of any frame
    std::vector<uint8_t> fr_ngrp;             // [nframes]
    std::vector<uint32_t> fr_gkey;            // [nframes][kMaxFrameGroups]
    std::vector<uint8_t> fr_grp;              // [nframes][P]
    std::vector<uint8_t> fr_order;            // [nframes][P] points sorted by group
    std::vector<uint8_t> fr_goff;             // [nframes][kMaxFrameGroups + 1] group offsets
    // Box tiles: the parent slots sorted by parent cone and cut into runs of
    // at most kBoxTile slots of one cone (boxes that share every frame), for
    // the child-to-parent kernel that batches boxes as matrix columns.
    int64_t ntiles = 0;
    std::vector<int32_t> bt_slot;             // [ntiles][kBoxTile] parent slot, -1 pad
    std::vector<int32_t> bt_frame;            // [ntiles][8] frame of octant o, -1 none
    std::vector<int32_t> slot_order;          // [nslots_{d-1}] parent slots in tile order
    // entries of the box tiles: (octant, group) pairs of the tile's frames in
    // octant order, with their child slot in each of the tile's boxes
    std::vector<int32_t> te_start;            // [ntiles + 1] first entry of the tile
    double te_per_tile = 0;                   // entries per tile, on average
    std::vector<uint16_t> te_go;              // [ntiles][9] first entry of octant o, relative; [8] = count
    std::vector<int32_t> te_info;             // [entries] g0 | cnt << 8 | o << 16
    std::vector<int32_t> te_cs;               // [entries][kBoxTile] child slot, -1 no child, -2 cone missing
    std::vector<uint8_t> te_mask;             // [ntiles][kBoxTile] children of the box (bit o)
    // Cousin-target pairs (levels d >= 3): for every target box T, cousin
    // c of T and target t of T, entry pair_base[T] + c * n_T + t holds the
    // slot of the cone of cousin c that contains t, t's local coordinates in
    // it and the centred factor G(x_t, x_c); built when they fit the budget.
    bool use_pairs = false;
    bool pairs_device = false;                // built in device memory (plan_gpu.hip), not here
    bool pairs_ordered = false;               // with the cone-ordered copy
    std::vector<int64_t> pair_base;           // [nbox + 1]
    std::vector<int32_t> pr_slot;             // [npairs]
    std::vector<double> pr_t;                 // [3][npairs] (structure of arrays)
    std::vector<double> pr_g;                 // [2][npairs]
    std::vector<int32_t> pr_order;            // pairs with a cone, ordered by slot (-1: padding)
    std::vector<int32_t> pro_slot;            // their slots, in that order
    std::vector<double> pro_t;                // [3][npairs with a cone], in that order
    std::vector<double> pro_g;                // [2][npairs with a cone], in that order
};

struct HostPlan {
    int64_t n = 0;
    double kappa = 0;
    int D = 0, ps = 3, pang = 5, P = 75;
    double H1 = 0, x1[3] = {0, 0, 0}, corner[3] = {0, 0, 0};
    std::vector<int32_t> perm;                // Morton position -> input index
    std::vector<double> pts;                  // [n][3] Morton order
    std::vector<HostLevel> L;                 // levels 0..D (0 unused)
    // adaptive octree (leaf_max > 0): the direct evaluations of every level-D
    // box as point ranges [near_lo, near_hi) of the leaves whose neighbourhood
    // holds it, on their own levels
    int leaf_max = 0;
    bool adaptive = false;
    std::vector<int32_t> near_start, near_lo, near_hi;
    ifgf_stats stats{};
};

// Marks and numbers the relevant cone segments of one level (rules (i) and
// (ii) of Sec. 3.3.2) in place of the host loop: fills hp.L[d]'s nslots,
// slot_start, slot_box, slot_cone, cell_base and cell_mask exactly as the
// host builder would, and adds the cones marked only by dilation to
// n_dilated.  Returns "" or a message (code set).
struct ConeMarker {
    virtual ~ConeMarker() = default;
    virtual std::string mark_level(HostPlan& hp, int d, bool dilate, int64_t& n_dilated, ifgf_status& code) = 0;
};
// The device implementation (plan_gpu.hip); uses the current GPU.
std::unique_ptr<ConeMarker> make_gpu_cone_marker();

// Builds the hierarchy; returns an empty string on success, else a message.
// `code` receives the ifgf_status on failure.
// tab_elem_bytes: device bytes of one tabulated cousin-target pair (0: none);
// ord_elem_bytes: device bytes of its cone-ordered copy (0: none);
// pair_budget: device bytes the pair tables may take.
// marker: numbers the relevant cones (null: on the host).
// pairs_device: the pair tables are left to build_pairs_device (only their
// offsets pair_base are built here).
// leaf_max: adaptive octree, boxes of level >= 2 with at most leaf_max points
// are not split (0: every leaf on level D).
std::string build_host_plan(const double* points, int64_t n, double kappa, int levels, int ps, int pang,
                            int leaf_ns, int leaf_nc, bool dilate, double tab_elem_bytes, double ord_elem_bytes,
                            double pair_budget, HostPlan& hp, ifgf_status& code, ConeMarker* marker = nullptr,
                            bool pairs_device = false, int leaf_max = 0);

// ---------------------------------------------------------- device mirror

struct LevelDev {
    int nbox, ns, nc, ncell, W, nslots;
    double H, h, ds, dang;                    // box side, circumradius, intervals
    const int32_t* box_start;
    const double* box_ctr;
    const uint8_t* box_oct;
    const int32_t* pt_box;
    const int32_t* chl_start;
    const int32_t* chl;
    const int32_t* nbr_start;
    const int32_t* nbr;
    const int32_t* cou_start;
    const int32_t* cou;
    // adaptive octree: slots of this level's leaf boxes (levels 3..D-1), and
    // on level D the direct evaluations as point ranges per box
    int nleaf_slots;
    const int32_t* leaf_slots;
    const int32_t* near_start;
    const int32_t* near_lo;
    const int32_t* near_hi;
    const int32_t* cell_base;
    const unsigned long long* cell_mask;
    const int32_t* slot_box;
    const int32_t* slot_cone;
    const double* node_r;
    const double* node_dir;
    // child-to-parent frames (children at this level); fr_t / fr_ratio are
    // float for the mixed path and double for FP64
    int use_frames;
    const int32_t* child_of;
    const int32_t* pframe;
    const uint32_t* fr_key;
    const void* fr_t;
    const void* fr_ratio;
    int frame_groups_ok;
    const uint8_t* fr_ngrp;
    const uint32_t* fr_gkey;
    const uint8_t* fr_grp;
    const uint8_t* fr_order;
    const uint8_t* fr_goff;
    int ntiles;
    const int32_t* bt_slot;
    const int32_t* bt_frame;
    const int32_t* slot_order;               // parent slots in tile order, or null
    const int32_t* te_start;                 // tile entries (see HostLevel), or null
    const uint16_t* te_go;
    const int32_t* te_info;
    const int32_t* te_cs;
    const uint8_t* te_mask;
    // cousin-target pairs (float for mixed, double for FP64)
    int use_pairs;
    long long npairs_cou;
    const long long* pair_base;
    const int32_t* pr_slot;
    const void* pr_t;
    const void* pr_g;
    long long npairs_ord;                     // entries of pr_order (0: no ordered copy)
    const int32_t* pr_order;
    const int32_t* pro_slot;
    const void* pro_t;
    const void* pro_g;
};

// Slot of cone (cell, i_s) of `box`, or -1 if it was not marked relevant.
__device__ inline int lookup(const LevelDev& L, int box, int cell, int is)
{
    size_t c = (size_t)box * L.ncell + cell;
    const unsigned long long* M = L.cell_mask + c * L.W;
    int w = is >> 6, bit = is & 63;
    unsigned long long m = M[w];
    if (!((m >> bit) & 1ull)) return -1;
    int cnt = __popcll(m & ((1ull << bit) - 1ull));
    for (int i = 0; i < w; ++i) cnt += __popcll(M[i]);
    return L.cell_base[c] + cnt;
}

struct KernelConsts {
    ChebNodes cs, ca;        // radial and angular node sets
    double kappa;            // wavenumber of the phases: k, or -k for the adjoint
    int n;                   // points
    unsigned long long* miss;  // device counter of interpolation misses
    int adj;                 // 1: the adjoint (conjugated centred factors and
                             // ratios); never inferred from the sign of kappa,
                             // which is -0.0 for the adjoint at k = 0
    int ps = 0, pa = 0;      // node counts P_s, P_ang (read by the kernels
                             // instantiated for run-time node counts)
};

// A plan: the host hierarchy, its device copy and the workspaces.
struct DevicePlan {
    HostPlan hp;
    int device = -1;
    int precision = IFGF_FP64;
    int max_nrhs = 16;
    // distinct targets: points [0, n_src) are the sources, [n_src, n_src +
    // n_tgt) the targets (densities zero there); n_tgt = 0: every point is both
    int64_t n_src = 0, n_tgt = 0;
    int store_levels = -1;
    bool host_only = false;
    size_t ws_limit = 0;
    // device hierarchy
    double* pts = nullptr;
    int32_t* perm = nullptr;    // Morton position -> input index
    int32_t* iperm = nullptr;   // input index -> Morton position
    std::vector<LevelDev> L;
    unsigned long long* miss = nullptr;
    void* zero_cone = nullptr;  // [P][kMaxRhsPass] complex zeros (FP32 view)
    int64_t max_pairs = 0;      // largest cousin-pair table of a level (0: none)
    // (target box, cousin, target) pair offsets of every level d >= 3 (device,
    // [nbox + 1]) and their counts, for the two-phase evaluation with
    // per-pair geometry where no pair table is kept
    const long long* pair_off[IFGF_MAX_LEVELS + 1] = {};
    int64_t npairs_all[IFGF_MAX_LEVELS + 1] = {};
    int64_t pval_pairs = 0;     // pairs the pval workspace holds
    // levels without a pair table: the pairs with a cone in cone order, each
    // as its target point (low 24 bits) and its cousin's index in the target
    // box's cousin list (high 8 bits), runs of one cone padded to kPairQuad
    // entries with 0xffffffff (null: not built)
    const uint32_t* go_ord[IFGF_MAX_LEVELS + 1] = {};
    int64_t ngo[IFGF_MAX_LEVELS + 1] = {};
    std::vector<void*> allocs;
    size_t tree_bytes = 0;
    // workspaces, sized for `ws_rb` right-hand sides per pass
    int ws_rb = 0;
    bool ws_store = false;
    void* dens_m = nullptr;     // [n][rb] complex, Morton order
    void* out_m = nullptr;      // [n][rb] complex, Morton order
    void* gout_m = nullptr;     // [n][rb] complex, Morton order (gradient input)
    double* grad_m = nullptr;   // [n][3] FP64, Morton order (gradient output)
    void* pval = nullptr;       // [max_pairs] complex: value of every cousin pair (one RHS)
    bool ws_store_pref = false; // keep the cone values of every level
    void* F[IFGF_MAX_LEVELS + 1] = {};  // cone values per level [nslots][P][rb]
    std::vector<void*> ws_allocs;
    size_t ws_bytes = 0;
    // stage timing (ifgf_plan_profile)
    bool profiling = false;
    std::vector<hipEvent_t> events;
    size_t next_event = 0;
    struct Pending { int stage, level; size_t e0, e1; };
    std::vector<Pending> pending;
    double stage_ms[IFGF_NUM_STAGES] = {};
    int64_t stage_launches[IFGF_NUM_STAGES] = {};
    // the same per level (stages of one level: cousin evaluation d, the
    // child-to-parent step from d; others at level 0)
    double level_ms[IFGF_NUM_STAGES][IFGF_MAX_LEVELS + 1] = {};
    int64_t level_launches[IFGF_NUM_STAGES][IFGF_MAX_LEVELS + 1] = {};
    // child-to-parent variant per (right-hand-side block 1 / 4 / 16, level),
    // -1: the default rule; set by ifgf_plan_autotune
    int c2p_choice[3][IFGF_MAX_LEVELS + 1];
    DevicePlan()
    {
        for (auto& r : c2p_choice)
            for (int& c : r) c = -1;
    }
    int tune_gen = 0;            // bumped when the choices change
    int ws_gen = 0;              // bumped when the workspaces are reallocated
    // second stream of an eager apply: the near field and the cousin
    // evaluations run on it beside the chain of child-to-parent steps,
    // ordered by events (created on first use)
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> sync_ev;   // [0] inputs permuted, [1] side done, then cone levels ready / read
    bool capturing = false;            // an apply graph is being captured
    bool no_alloc = false;             // ifgf_apply_noalloc: one stream, scratch workspaces
    // captured apply graphs (use_graph)
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    struct GraphEntry {
        const void* a; void* out; int nrhs; bool adj; int ws_gen, tune_gen; hipGraphExec_t exec; uint64_t used;
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    // stream of the last apply or gradient call (synchronised by ifgf_plan_check)
    hipStream_t last_stream = nullptr;
    // every stream that ran work on the plan's workspaces since they were last
    // (re)allocated: the work a reallocation or the plan's release waits for
    std::vector<hipStream_t> used_streams;
    void use_stream(hipStream_t st)
    {
        last_stream = st;
        for (hipStream_t u : used_streams)
            if (u == st) return;
        used_streams.push_back(st);
    }
    // what the stored cone values hold (for gradient reuse)
    const void* stored_dens = nullptr;
    int stored_nrhs = 0;
    bool stored_valid = false;
};

// Records a HIP event pair around one kernel launch when profiling is on.
class StageTimer {
  public:
    StageTimer(DevicePlan& p, int stage, hipStream_t st, int level = 0) : p_(p), stage_(stage), level_(level), st_(st)
    {
        if (p_.profiling) e0_ = record();
    }
    ~StageTimer()
    {
        if (p_.profiling && e0_ != (size_t)-1) {
            size_t e1 = record();
            if (e1 != (size_t)-1) p_.pending.push_back({stage_, level_, e0_, e1});
        }
    }

  private:
    size_t record()
    {
        if (p_.next_event == p_.events.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return (size_t)-1;
            p_.events.push_back(e);
        }
        size_t i = p_.next_event++;
        if (hipEventRecord(p_.events[i], st_) != hipSuccess) return (size_t)-1;
        return i;
    }
    DevicePlan& p_;
    int stage_, level_;
    hipStream_t st_;
    size_t e0_ = (size_t)-1;
};

// Kernel pipeline entry points (kernels.hip).  `adj` selects the adjoint
// (windows swapped, kernel conjugated).  Each enqueues on `stream` and
// returns hipSuccess or the first launch error.
hipError_t run_apply(DevicePlan& p, const void* dens, int nrhs, void* out, bool adj, hipStream_t stream);
// Level d's cousin-target pair table (and with `ordered` its cone-ordered
// copy) computed in device memory from the uploaded level (plan_gpu.hip).
hipError_t build_pairs_device(DevicePlan& p, int d, bool ordered);
// Level d's pairs (of a level without a pair table) in cone order, as
// go_ord[d] / ngo[d] (plan_gpu.hip).  Leaves go_ord[d] null where a pair has
// no cone, where the points or cousin lists do not fit the packing, or
// where `budget` bytes would not hold the order.
hipError_t build_pair_order_device(DevicePlan& p, int d, double budget);
// Allocates the workspaces an apply with nrhs right-hand sides needs (so
// that the apply itself allocates nothing and can be captured).
hipError_t run_prepare(DevicePlan& p, int nrhs);
// Records after an apply (eager or replayed) what the stored cone values hold.
void note_apply(DevicePlan& p, const void* dens, int nrhs, bool adj);
// Times every child-to-parent variant of every level for nrhs right-hand
// sides (densities zero, synchronous) and keeps the fastest.
hipError_t run_autotune(DevicePlan& p, int nrhs, hipStream_t st);
// Variant of level d for nrhs right-hand sides (-1: no child-to-parent step).
int kernel_choice(const DevicePlan& p, int nrhs, int d);
// Variants applicable at level d for nrhs right-hand sides (count; v gets
// up to kC2PVariants entries).
int kernel_candidates(const DevicePlan& p, int nrhs, int d, int* v);
// Sets (variant >= 0) or resets (-1) the variant of level d; false if the
// variant does not apply there.
bool set_kernel_choice(DevicePlan& p, int nrhs, int d, int variant);
hipError_t run_grad(DevicePlan& p, const void* dens, const void* gout, int nrhs, double* grad, bool reuse,
                    hipStream_t stream);
// The apply with its workspaces in the library's static per-GPU scratch
// array (no allocation, everything on `stream`); hipErrorOutOfMemory when
// they do not fit in scratch_bytes().
hipError_t run_apply_noalloc(DevicePlan& p, const void* dens, int nrhs, void* out, bool adj, hipStream_t stream);
// Takes the current device's scratch address (once per device).
hipError_t scratch_init(int device);
// Waits for the plan's work on every stream that ran it since its workspaces
// were last (re)allocated, and on its own streams (not the whole device).
hipError_t wait_plan_streams(DevicePlan& p);
size_t scratch_bytes();
// Scratch bytes an apply of nrhs right-hand sides needs in that mode.
size_t noalloc_bytes(const DevicePlan& p, int nrhs);

}  // namespace ifgf
