// C ABI of the IFGF library (declared in include/ifgf.h).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ifgf_internal.hpp"

struct ifgf_plan {
    ifgf::DevicePlan p;
};

namespace {

thread_local std::string g_last_error;

ifgf_status fail(ifgf_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

ifgf_status hip_fail(hipError_t e, const char* where)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(IFGF_E_OUT_OF_MEMORY, std::string(where) + ": " + hipGetErrorString(e));
    return fail(IFGF_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

template <typename T>
hipError_t upload(ifgf::DevicePlan& p, const std::vector<T>& v, const T** out)
{
    *out = nullptr;
    if (v.empty()) return hipSuccess;
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    p.allocs.push_back(d);
    p.tree_bytes += v.size() * sizeof(T);
    e = hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    *out = (const T*)d;
    return e;
}

void release(ifgf::DevicePlan& p)
{
    if (p.device >= 0) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p.device);
        // the plan's work on every stream that used it (not the whole device)
        (void)ifgf::wait_plan_streams(p);
        for (void* q : p.ws_allocs) (void)hipFree(q);
        for (void* q : p.allocs) (void)hipFree(q);
        for (hipEvent_t ev : p.events) (void)hipEventDestroy(ev);
        for (hipEvent_t ev : p.sync_ev) (void)hipEventDestroy(ev);
        for (auto& g : p.graphs) (void)hipGraphExecDestroy(g.exec);
        if (p.cap_stream) (void)hipStreamDestroy(p.cap_stream);
        if (p.side) (void)hipStreamDestroy(p.side);
        if (cur >= 0) (void)hipSetDevice(cur);
    }
    p.graphs.clear();
    p.cap_stream = nullptr;
    p.side = nullptr;
    p.sync_ev.clear();
    p.ws_allocs.clear();
    p.allocs.clear();
    p.events.clear();
}

hipError_t upload_plan(ifgf::DevicePlan& p)
{
    using namespace ifgf;
    HostPlan& hp = p.hp;
    hipError_t e;
    const double* dp = nullptr;
    const int32_t* ip = nullptr;
    if ((e = upload(p, hp.pts, &dp)) != hipSuccess) return e;
    p.pts = const_cast<double*>(dp);
    if ((e = upload(p, hp.perm, &ip)) != hipSuccess) return e;
    p.perm = const_cast<int32_t*>(ip);
    std::vector<int32_t> iperm(hp.n);
    for (int64_t i = 0; i < hp.n; ++i) iperm[hp.perm[i]] = (int32_t)i;
    if ((e = upload(p, iperm, &ip)) != hipSuccess) return e;
    p.iperm = const_cast<int32_t*>(ip);
    void* m = nullptr;
    if ((e = hipMalloc(&m, sizeof(unsigned long long))) != hipSuccess) return e;
    p.allocs.push_back(m);
    p.miss = (unsigned long long*)m;
    if ((e = hipMemset(m, 0, sizeof(unsigned long long))) != hipSuccess) return e;
    // zeros for one cone of kMaxRhsPass right-hand sides in the widest type
    const size_t zb = (size_t)hp.P * kMaxRhsPass * 2 * sizeof(double);
    if ((e = hipMalloc(&m, zb)) != hipSuccess) return e;
    p.allocs.push_back(m);
    p.zero_cone = m;
    if ((e = hipMemset(m, 0, zb)) != hipSuccess) return e;
    p.L.assign(hp.D + 1, LevelDev{});
    // device bytes the cone orders of the levels without pair tables may
    // take (IFGF_GEO_ORDER_BUDGET_MB, default 16384; 0: none)
    double geo_order_budget = 16384.0 * 1024.0 * 1024.0;
    if (const char* v = std::getenv("IFGF_GEO_ORDER_BUDGET_MB")) geo_order_budget = std::atof(v) * 1024.0 * 1024.0;
    for (int d = 1; d <= hp.D; ++d) {
        HostLevel& H = hp.L[d];
        LevelDev& L = p.L[d];
        L.nbox = (int)H.nbox;
        L.ns = H.ns;
        L.nc = H.nc;
        L.ncell = H.ncell;
        L.W = H.W;
        L.nslots = (int)H.nslots;
        L.H = H.H;
        L.h = H.h;
        L.ds = H.ds;
        L.dang = H.dang;
        bool interp_level = d >= 3;
        bool parent_of_interp = d >= 3 && d < hp.D;
        if (d == hp.D || interp_level) {
            if ((e = upload(p, H.box_start, &L.box_start)) != hipSuccess) return e;
            if ((e = upload(p, H.box_ctr, &L.box_ctr)) != hipSuccess) return e;
            if ((e = upload(p, H.pt_box, &L.pt_box)) != hipSuccess) return e;
        }
        if (d == hp.D)
            if ((e = upload(p, H.nbr_start, &L.nbr_start)) != hipSuccess || (e = upload(p, H.nbr, &L.nbr)) != hipSuccess)
                return e;
        // adaptive octree: direct evaluations as point ranges (level D) and
        // the slots of the leaf boxes above level D
        if (hp.adaptive && d == hp.D) {
            if ((e = upload(p, hp.near_start, &L.near_start)) != hipSuccess) return e;
            if ((e = upload(p, hp.near_lo, &L.near_lo)) != hipSuccess) return e;
            if ((e = upload(p, hp.near_hi, &L.near_hi)) != hipSuccess) return e;
        }
        if (hp.adaptive && d >= 3 && d < hp.D) {
            L.nleaf_slots = (int)H.leaf_slots.size();
            if ((e = upload(p, H.leaf_slots, &L.leaf_slots)) != hipSuccess) return e;
        }
        if (interp_level) {
            if ((e = upload(p, H.box_oct, &L.box_oct)) != hipSuccess) return e;
            if ((e = upload(p, H.cou_start, &L.cou_start)) != hipSuccess) return e;
            if ((e = upload(p, H.cou, &L.cou)) != hipSuccess) return e;
            if ((e = upload(p, H.cell_base, &L.cell_base)) != hipSuccess) return e;
            const uint64_t* mk = nullptr;
            if ((e = upload(p, H.cell_mask, &mk)) != hipSuccess) return e;
            L.cell_mask = (const unsigned long long*)mk;
            if ((e = upload(p, H.slot_box, &L.slot_box)) != hipSuccess) return e;
            if ((e = upload(p, H.slot_cone, &L.slot_cone)) != hipSuccess) return e;
            if ((e = upload(p, H.node_r, &L.node_r)) != hipSuccess) return e;
            if ((e = upload(p, H.node_dir, &L.node_dir)) != hipSuccess) return e;
        }
        if (parent_of_interp) {
            if ((e = upload(p, H.chl_start, &L.chl_start)) != hipSuccess) return e;
        }
        if (interp_level) {
            // pair offsets of every level (the two-phase cousin evaluation)
            std::vector<long long> off(H.nbox + 1, 0);
            for (int64_t T = 0; T < H.nbox; ++T)
                off[T + 1] = off[T] + (long long)(H.box_start[T + 1] - H.box_start[T]) *
                                          (H.cou_start[T + 1] - H.cou_start[T]);
            p.npairs_all[d] = off[H.nbox];
            const long long* po = nullptr;
            if ((e = upload(p, off, &po)) != hipSuccess) return e;
            p.pair_off[d] = po;
            // without a cone-ordered pair table: the pairs in cone order, for the
            // matrix-core evaluation of batched right-hand sides
            if (!(H.use_pairs && H.pairs_ordered) && p.max_nrhs >= 4 && geo_order_budget > 0) {
                if ((e = build_pair_order_device(p, d, geo_order_budget)) != hipSuccess) return e;
                geo_order_budget -= 4.0 * (double)p.ngo[d];
            }
        }
        L.use_pairs = H.use_pairs ? 1 : 0;
        if (H.use_pairs && H.pairs_device) {
            // computed in device memory from this level's tables (uploaded above)
            if ((e = build_pairs_device(p, d, H.pairs_ordered)) != hipSuccess) return e;
            p.max_pairs = std::max<int64_t>(p.max_pairs, (int64_t)H.pair_base[H.nbox]);
        } else if (H.use_pairs) {
            L.npairs_cou = (long long)H.pr_slot.size();
            std::vector<long long> pb(H.pair_base.begin(), H.pair_base.end());
            if ((e = upload(p, pb, &L.pair_base)) != hipSuccess) return e;
            if ((e = upload(p, H.pr_slot, &L.pr_slot)) != hipSuccess) return e;
            L.npairs_ord = (long long)H.pr_order.size();
            if (L.npairs_ord > 0) {
                if ((e = upload(p, H.pr_order, &L.pr_order)) != hipSuccess) return e;
                if ((e = upload(p, H.pro_slot, &L.pro_slot)) != hipSuccess) return e;
                if (p.precision == IFGF_MIXED) {
                    std::vector<float> t(H.pro_t.begin(), H.pro_t.end()), g(H.pro_g.begin(), H.pro_g.end());
                    const float* dt = nullptr;
                    if ((e = upload(p, t, &dt)) != hipSuccess) return e;
                    L.pro_t = dt;
                    if ((e = upload(p, g, &dt)) != hipSuccess) return e;
                    L.pro_g = dt;
                } else {
                    const double* dt = nullptr;
                    if ((e = upload(p, H.pro_t, &dt)) != hipSuccess) return e;
                    L.pro_t = dt;
                    if ((e = upload(p, H.pro_g, &dt)) != hipSuccess) return e;
                    L.pro_g = dt;
                }
            }
            p.max_pairs = std::max<int64_t>(p.max_pairs, (int64_t)H.pr_slot.size());
            if (p.precision == IFGF_MIXED) {
                std::vector<float> t(H.pr_t.begin(), H.pr_t.end()), g(H.pr_g.begin(), H.pr_g.end());
                const float* dt = nullptr;
                if ((e = upload(p, t, &dt)) != hipSuccess) return e;
                L.pr_t = dt;
                if ((e = upload(p, g, &dt)) != hipSuccess) return e;
                L.pr_g = dt;
            } else {
                const double* dt = nullptr;
                if ((e = upload(p, H.pr_t, &dt)) != hipSuccess) return e;
                L.pr_t = dt;
                if ((e = upload(p, H.pr_g, &dt)) != hipSuccess) return e;
                L.pr_g = dt;
            }
            std::vector<double>().swap(H.pr_t);
            std::vector<double>().swap(H.pr_g);
            std::vector<int32_t>().swap(H.pr_slot);
            std::vector<int32_t>().swap(H.pr_order);
            std::vector<int32_t>().swap(H.pro_slot);
            std::vector<double>().swap(H.pro_t);
            std::vector<double>().swap(H.pro_g);
        }
        L.use_frames = H.use_frames ? 1 : 0;
        if (d >= 4)
            if ((e = upload(p, H.child_of, &L.child_of)) != hipSuccess) return e;
        if (d >= 4 && H.use_frames) {
            if ((e = upload(p, H.pframe, &L.pframe)) != hipSuccess) return e;
            if ((e = upload(p, H.fr_key, &L.fr_key)) != hipSuccess) return e;
            if (p.precision == IFGF_MIXED) {
                std::vector<float> t(H.fr_t.begin(), H.fr_t.end()), r(H.fr_ratio.begin(), H.fr_ratio.end());
                const float* dt = nullptr;
                if ((e = upload(p, t, &dt)) != hipSuccess) return e;
                L.fr_t = dt;
                if ((e = upload(p, r, &dt)) != hipSuccess) return e;
                L.fr_ratio = dt;
            } else {
                const double* dt = nullptr;
                if ((e = upload(p, H.fr_t, &dt)) != hipSuccess) return e;
                L.fr_t = dt;
                if ((e = upload(p, H.fr_ratio, &dt)) != hipSuccess) return e;
                L.fr_ratio = dt;
            }
            L.frame_groups_ok = H.frame_groups_ok ? 1 : 0;
            if (H.frame_groups_ok) {
                if ((e = upload(p, H.fr_ngrp, &L.fr_ngrp)) != hipSuccess) return e;
                if ((e = upload(p, H.fr_gkey, &L.fr_gkey)) != hipSuccess) return e;
                if ((e = upload(p, H.fr_grp, &L.fr_grp)) != hipSuccess) return e;
                if ((e = upload(p, H.fr_order, &L.fr_order)) != hipSuccess) return e;
                if ((e = upload(p, H.fr_goff, &L.fr_goff)) != hipSuccess) return e;
                L.ntiles = (int)H.ntiles;
                if ((e = upload(p, H.bt_slot, &L.bt_slot)) != hipSuccess) return e;
                if ((e = upload(p, H.bt_frame, &L.bt_frame)) != hipSuccess) return e;
                if ((int64_t)H.slot_order.size() == hp.L[d - 1].nslots && !H.slot_order.empty())
                    if ((e = upload(p, H.slot_order, &L.slot_order)) != hipSuccess) return e;
                if (!H.te_start.empty() && !H.te_info.empty()) {
                    if ((e = upload(p, H.te_start, &L.te_start)) != hipSuccess) return e;
                    if ((e = upload(p, H.te_go, &L.te_go)) != hipSuccess) return e;
                    if ((e = upload(p, H.te_info, &L.te_info)) != hipSuccess) return e;
                    if ((e = upload(p, H.te_cs, &L.te_cs)) != hipSuccess) return e;
                    if ((e = upload(p, H.te_mask, &L.te_mask)) != hipSuccess) return e;
                }
                std::vector<int32_t>().swap(H.te_cs);
                std::vector<int32_t>().swap(H.te_info);
            }
            // the host copies are no longer needed
            std::vector<double>().swap(H.fr_t);
            std::vector<double>().swap(H.fr_ratio);
        }
    }
    return hipSuccess;
}

ifgf_status check_apply_args(ifgf_plan_t plan, const void* a, const void* out, int32_t nrhs)
{
    if (!plan) return fail(IFGF_E_INVALID_ARG, "plan is NULL");
    if (plan->p.host_only) return fail(IFGF_E_UNSUPPORTED, "plan was created with host_only");
    if (!a || !out) return fail(IFGF_E_INVALID_ARG, "NULL device pointer");
    if (a == out) return fail(IFGF_E_INVALID_ARG, "input and output must not alias");
    if (nrhs < 1 || nrhs > plan->p.max_nrhs)
        return fail(IFGF_E_INVALID_ARG, "nrhs must be in [1, max_nrhs=" + std::to_string(plan->p.max_nrhs) + "]");
    return IFGF_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

static ifgf_status create_common(const double* points, int64_t n, int64_t n_tgt, double k, int32_t levels,
                                 const int32_t* degrees, const ifgf_options* opt, ifgf_plan_t* plan)
{
    if (!plan) return fail(IFGF_E_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    ifgf_options o{};
    if (opt) o = *opt;
    int ps = degrees ? degrees[0] : 3, pa = degrees ? degrees[1] : 5;
    if (ps < 1 || pa < 1) return fail(IFGF_E_INVALID_ARG, "degrees (node counts) must be >= 1");
    if (ps > ifgf::kMaxNodes || pa > ifgf::kMaxNodes)
        return fail(IFGF_E_UNSUPPORTED, "degrees (node counts) above 8 are not supported");
    // {3,5}, {4,6} and {2,3} have kernels compiled for their node counts;
    // other counts run the kernels that read them at run time, which compute
    // the cousin geometry per evaluation (no pair tables)
    const bool compiled = (ps == 3 && pa == 5) || (ps == 4 && pa == 6) || (ps == 2 && pa == 3);
    int leaf_ns = o.leaf_ns ? o.leaf_ns : 1, leaf_nc = o.leaf_nc ? o.leaf_nc : 2;
    if (o.precision != IFGF_FP64 && o.precision != IFGF_MIXED) return fail(IFGF_E_INVALID_ARG, "unknown precision");
    int max_nrhs = o.max_nrhs ? o.max_nrhs : 16;
    if (max_nrhs < 1 || max_nrhs > 4096) return fail(IFGF_E_INVALID_ARG, "max_nrhs must be in [1, 4096]");
    ifgf_plan* pl = new (std::nothrow) ifgf_plan();
    if (!pl) return fail(IFGF_E_OUT_OF_MEMORY, "host allocation failed");
    ifgf::DevicePlan& p = pl->p;
    p.precision = o.precision;
    p.max_nrhs = max_nrhs;
    p.store_levels = o.store_levels;
    p.host_only = o.host_only != 0;
    p.use_graph = o.use_graph != 0;
    p.ws_limit = o.workspace_limit;
    p.n_tgt = n_tgt;
    p.n_src = n - n_tgt;
    ifgf_status code = IFGF_OK;
    std::string msg;
    try {
        // a tabulated cousin-target pair: slot, 3 local coordinates, complex G
        double pair_bytes = p.host_only || !compiled ? 0.0 : (o.precision == IFGF_MIXED ? 24.0 : 44.0);
        double ord_bytes = p.host_only || !compiled ? 0.0 : (o.precision == IFGF_MIXED ? 28.0 : 48.0);
        // pair tables: IFGF_PAIR_BUDGET_MB, else a quarter of the free device
        // memory, at most 64 GiB
        double budget = 0.0;
        if (const char* env = std::getenv("IFGF_PAIR_BUDGET_MB")) {
            budget = std::atof(env) * 1024.0 * 1024.0;
        } else if (!p.host_only) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) == hipSuccess) budget = std::min(0.25 * (double)fr, 64.0 * (1ull << 30));
        }
        // relevant cones and pair tables on the GPU (IFGF_HOST_PLAN=1: on the host)
        std::unique_ptr<ifgf::ConeMarker> marker;
        const char* hv = std::getenv("IFGF_HOST_PLAN");
        const bool on_gpu = !p.host_only && !(hv && std::atoi(hv) != 0);
        if (on_gpu) marker = ifgf::make_gpu_cone_marker();
        msg = ifgf::build_host_plan(points, n, k, levels, ps, pa, leaf_ns, leaf_nc, o.no_dilate == 0, pair_bytes,
                                    ord_bytes, budget, p.hp, code, marker.get(), on_gpu, o.leaf_max);
    } catch (const std::bad_alloc&) {
        delete pl;
        return fail(IFGF_E_OUT_OF_MEMORY, "host allocation failed while building the plan");
    } catch (const std::exception& ex) {
        delete pl;
        return fail(IFGF_E_INTERNAL, ex.what());
    }
    if (code != IFGF_OK) {
        delete pl;
        return fail(code, msg);
    }
    if (!p.host_only) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) {
            delete pl;
            return hip_fail(e, "hipGetDevice");
        }
        p.device = dev;
        // the device's scratch address for ifgf_apply_noalloc, taken at set-up
        // (once per device, with the plan's device current)
        e = ifgf::scratch_init(dev);
        if (e != hipSuccess) {
            delete pl;
            return hip_fail(e, "taking the address of the device scratch array");
        }
        e = upload_plan(p);
        if (e != hipSuccess) {
            release(p);
            delete pl;
            return hip_fail(e, "uploading the plan");
        }
        if (p.ws_limit && p.tree_bytes > p.ws_limit) {
            release(p);
            delete pl;
            return fail(IFGF_E_OUT_OF_MEMORY, "workspace_limit is smaller than the hierarchy");
        }
        // keep every level's cone values when asked, or when they fit in a
        // quarter of the free device memory
        size_t total = 0;
        int rb = max_nrhs >= 5 ? 16 : (max_nrhs >= 2 ? 4 : 1);
        size_t ce = p.precision == IFGF_MIXED ? 8 : 16;
        for (int d = 3; d <= p.hp.D; ++d) total += (size_t)p.hp.L[d].nslots * p.hp.P * rb * ce;
        if (p.store_levels == 1) p.ws_store_pref = true;
        else if (p.store_levels == 0) p.ws_store_pref = false;
        else {
            size_t fr = 0, tot = 0;
            (void)hipMemGetInfo(&fr, &tot);
            p.ws_store_pref = total <= fr / 4 && (!p.ws_limit || p.tree_bytes + 2 * total <= p.ws_limit);
        }
    }
    p.hp.stats.device_bytes = (int64_t)p.tree_bytes;
    p.hp.stats.n_sources = p.n_tgt > 0 ? p.n_src : n;
    p.hp.stats.n_targets = p.n_tgt > 0 ? p.n_tgt : n;
    *plan = pl;
    return IFGF_OK;
}

ifgf_status ifgf_plan_create(const double* points, int64_t n, double k, int32_t levels, const int32_t* degrees,
                             const ifgf_options* opt, ifgf_plan_t* plan)
{
    return create_common(points, n, 0, k, levels, degrees, opt, plan);
}

ifgf_status ifgf_plan_create_targets(const double* sources, int64_t n, const double* targets, int64_t m, double k,
                                     int32_t levels, const int32_t* degrees, const ifgf_options* opt,
                                     ifgf_plan_t* plan)
{
    if (!plan) return fail(IFGF_E_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (!sources || !targets) return fail(IFGF_E_INVALID_ARG, "sources or targets is NULL");
    if (n < 1 || m < 1) return fail(IFGF_E_INVALID_ARG, "need at least one source and one target");
    if (n + m > (int64_t)INT32_MAX / 2) return fail(IFGF_E_INVALID_ARG, "too many points for 32-bit indexing");
    std::vector<double> all;
    try {
        all.resize((size_t)3 * (n + m));
    } catch (const std::bad_alloc&) {
        return fail(IFGF_E_OUT_OF_MEMORY, "host allocation failed");
    }
    std::memcpy(all.data(), sources, sizeof(double) * 3 * (size_t)n);
    std::memcpy(all.data() + 3 * n, targets, sizeof(double) * 3 * (size_t)m);
    return create_common(all.data(), n + m, m, k, levels, degrees, opt, plan);
}

// The apply as a captured graph: captured on the plan's own stream the first
// time a (densities, out, nrhs, direction) combination is seen with the
// current workspaces and kernel choices, then replayed on the caller's
// stream.  The graph holds kernel launches only.
static hipError_t apply_graph(ifgf::DevicePlan& p, const void* a, int nrhs, void* out, bool adj,
                              hipStream_t st)
{
    hipError_t e = ifgf::run_prepare(p, nrhs);
    if (e != hipSuccess) return e;
    ifgf::DevicePlan::GraphEntry* hit = nullptr;
    for (auto& g : p.graphs)
        if (g.a == a && g.out == out && g.nrhs == nrhs && g.adj == adj && g.ws_gen == p.ws_gen &&
            g.tune_gen == p.tune_gen)
            hit = &g;
    if (!hit) {
        if (!p.cap_stream && (e = hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return e;
        if ((e = hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
        p.capturing = true;
        hipError_t ea = ifgf::run_apply(p, a, nrhs, out, adj, p.cap_stream);
        p.capturing = false;
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(p.cap_stream, &graph);
        if (ea != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return ea != hipSuccess ? ea : e;
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        const size_t kMaxGraphs = 8;
        if (p.graphs.size() >= kMaxGraphs) {
            size_t old = 0;
            for (size_t i = 1; i < p.graphs.size(); ++i)
                if (p.graphs[i].used < p.graphs[old].used) old = i;
            (void)hipGraphExecDestroy(p.graphs[old].exec);
            p.graphs.erase(p.graphs.begin() + (long)old);
        }
        p.graphs.push_back({a, out, nrhs, adj, p.ws_gen, p.tune_gen, exec, 0});
        hit = &p.graphs.back();
    }
    hit->used = ++p.graph_clock;
    if ((e = hipGraphLaunch(hit->exec, st)) != hipSuccess) return e;
    ifgf::note_apply(p, a, nrhs, adj);
    return hipSuccess;
}

static ifgf_status apply_common(ifgf_plan_t plan, const void* a, int32_t nrhs, void* out, void* stream, bool adj)
{
    ifgf_status s = check_apply_args(plan, a, out, nrhs);
    if (s != IFGF_OK) return s;
    ifgf::DevicePlan& p = plan->p;
    DeviceGuard g(p.device);
    p.use_stream((hipStream_t)stream);
    hipError_t e = p.use_graph && !p.profiling ? apply_graph(p, a, nrhs, out, adj, (hipStream_t)stream)
                                               : ifgf::run_apply(p, a, nrhs, out, adj, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, adj ? "ifgf_apply_adjoint" : "ifgf_apply");
    return IFGF_OK;
}

ifgf_status ifgf_plan_autotune(ifgf_plan_t plan, int32_t nrhs, void* stream)
{
    if (!plan) return fail(IFGF_E_INVALID_ARG, "plan is NULL");
    if (plan->p.host_only) return fail(IFGF_E_UNSUPPORTED, "plan was created with host_only");
    if (nrhs < 1 || nrhs > plan->p.max_nrhs) return fail(IFGF_E_INVALID_ARG, "nrhs out of range");
    ifgf::DevicePlan& p = plan->p;
    DeviceGuard g(p.device);
    p.use_stream((hipStream_t)stream);
    hipError_t e = ifgf::run_autotune(p, nrhs, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ifgf_plan_autotune");
    return IFGF_OK;
}

ifgf_status ifgf_plan_set_kernel_choice(ifgf_plan_t plan, int32_t nrhs, const int32_t* variant)
{
    if (!plan || !variant) return fail(IFGF_E_INVALID_ARG, "NULL argument");
    if (nrhs < 1) return fail(IFGF_E_INVALID_ARG, "nrhs out of range");
    if (plan->p.host_only) return fail(IFGF_E_UNSUPPORTED, "plan was created with host_only");
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d)
        if (variant[d] >= 0 && ifgf::kernel_choice(plan->p, nrhs, d) < 0)
            return fail(IFGF_E_INVALID_ARG, "level has no child-to-parent step");
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d)
        if (variant[d] >= ifgf::kC2PVariants || variant[d] < -1)
            return fail(IFGF_E_INVALID_ARG, "unknown kernel variant");
    // validate all levels first, then set, so a failed call changes nothing
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) {
        if (variant[d] < 0) continue;
        int v[ifgf::kC2PVariants];
        const int n = ifgf::kernel_candidates(plan->p, nrhs, d, v);
        bool ok = false;
        for (int i = 0; i < n; ++i) ok = ok || v[i] == variant[d];
        if (!ok) return fail(IFGF_E_INVALID_ARG, "kernel variant does not apply at this level");
    }
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) (void)ifgf::set_kernel_choice(plan->p, nrhs, d, variant[d]);
    ++plan->p.tune_gen;
    return IFGF_OK;
}

ifgf_status ifgf_plan_kernel_candidates(ifgf_plan_t plan, int32_t nrhs, int32_t* mask)
{
    if (!plan || !mask) return fail(IFGF_E_INVALID_ARG, "NULL argument");
    if (nrhs < 1) return fail(IFGF_E_INVALID_ARG, "nrhs out of range");
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) {
        int v[ifgf::kC2PVariants];
        const int n = ifgf::kernel_candidates(plan->p, nrhs, d, v);
        int32_t m = 0;
        for (int i = 0; i < n; ++i) m |= 1 << v[i];
        mask[d] = m;
    }
    return IFGF_OK;
}

ifgf_status ifgf_plan_kernel_choice(ifgf_plan_t plan, int32_t nrhs, int32_t* variant)
{
    if (!plan || !variant) return fail(IFGF_E_INVALID_ARG, "NULL argument");
    if (nrhs < 1) return fail(IFGF_E_INVALID_ARG, "nrhs out of range");
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) variant[d] = ifgf::kernel_choice(plan->p, nrhs, d);
    return IFGF_OK;
}

ifgf_status ifgf_apply(ifgf_plan_t plan, const void* densities, int32_t nrhs, void* out, void* stream)
{
    return apply_common(plan, densities, nrhs, out, stream, false);
}

ifgf_status ifgf_apply_adjoint(ifgf_plan_t plan, const void* v, int32_t nrhs, void* out, void* stream)
{
    return apply_common(plan, v, nrhs, out, stream, true);
}

ifgf_status ifgf_apply_noalloc(ifgf_plan_t plan, const void* densities, int32_t nrhs, void* out, void* stream)
{
    ifgf_status s = check_apply_args(plan, densities, out, nrhs);
    if (s != IFGF_OK) return s;
    ifgf::DevicePlan& p = plan->p;
    const size_t need = ifgf::noalloc_bytes(p, nrhs), have = ifgf::scratch_bytes();
    if (need > have)
        return fail(IFGF_E_INVALID_ARG, "ifgf_apply_noalloc: the workspaces of this plan and nrhs need " +
                                            std::to_string(need) + " bytes, more than the " + std::to_string(have) +
                                            "-byte device scratch array; use ifgf_apply");
    DeviceGuard g(p.device);
    p.use_stream((hipStream_t)stream);
    hipError_t e = ifgf::run_apply_noalloc(p, densities, nrhs, out, false, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ifgf_apply_noalloc");
    return IFGF_OK;
}

static ifgf_status grad_common(ifgf_plan_t plan, const void* densities, const void* grad_out, int32_t nrhs,
                               double* grad_xyz, void* stream, bool reuse)
{
    ifgf_status s = check_apply_args(plan, densities, grad_xyz, nrhs);
    if (s != IFGF_OK) return s;
    if (!grad_out) return fail(IFGF_E_INVALID_ARG, "grad_out is NULL");
    ifgf::DevicePlan& p = plan->p;
    DeviceGuard g(p.device);
    p.use_stream((hipStream_t)stream);
    hipError_t e = ifgf::run_grad(p, densities, grad_out, nrhs, grad_xyz, reuse, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, reuse ? "ifgf_grad_targets_stored" : "ifgf_grad_targets");
    return IFGF_OK;
}

ifgf_status ifgf_grad_targets(ifgf_plan_t plan, const void* densities, const void* grad_out, int32_t nrhs,
                              double* grad_xyz, void* stream)
{
    return grad_common(plan, densities, grad_out, nrhs, grad_xyz, stream, false);
}

ifgf_status ifgf_grad_targets_stored(ifgf_plan_t plan, const void* densities, const void* grad_out, int32_t nrhs,
                                     double* grad_xyz, void* stream)
{
    return grad_common(plan, densities, grad_out, nrhs, grad_xyz, stream, true);
}

ifgf_status ifgf_plan_stats(ifgf_plan_t plan, ifgf_stats* out)
{
    if (!plan || !out) return fail(IFGF_E_INVALID_ARG, "NULL argument");
    *out = plan->p.hp.stats;
    out->device_bytes = (int64_t)(plan->p.tree_bytes + plan->p.ws_bytes);
    return IFGF_OK;
}

ifgf_status ifgf_plan_check(ifgf_plan_t plan, int64_t* misses)
{
    if (!plan || !misses) return fail(IFGF_E_INVALID_ARG, "NULL argument");
    *misses = 0;
    if (plan->p.host_only) return IFGF_OK;
    DeviceGuard g(plan->p.device);
    // the plan's last stream and its side stream (not the whole device)
    hipError_t e = hipStreamSynchronize(plan->p.last_stream);
    if (e == hipSuccess && plan->p.side) e = hipStreamSynchronize(plan->p.side);
    if (e != hipSuccess) return hip_fail(e, "ifgf_plan_check");
    unsigned long long m = 0;
    e = hipMemcpy(&m, plan->p.miss, sizeof(m), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "ifgf_plan_check");
    *misses = (int64_t)m;
    return IFGF_OK;
}

ifgf_status ifgf_plan_profile(ifgf_plan_t plan, int32_t enable)
{
    if (!plan) return fail(IFGF_E_INVALID_ARG, "plan is NULL");
    ifgf::DevicePlan& p = plan->p;
    if (p.host_only) return fail(IFGF_E_UNSUPPORTED, "plan was created with host_only");
    DeviceGuard g(p.device);
    if (enable) {
        hipError_t e = hipStreamSynchronize(p.last_stream);
        if (e == hipSuccess && p.side) e = hipStreamSynchronize(p.side);
        if (e != hipSuccess) return hip_fail(e, "ifgf_plan_profile");
        p.pending.clear();
        p.next_event = 0;
        for (int i = 0; i < IFGF_NUM_STAGES; ++i) {
            p.stage_ms[i] = 0.0;
            p.stage_launches[i] = 0;
            for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) {
                p.level_ms[i][d] = 0.0;
                p.level_launches[i][d] = 0;
            }
        }
    }
    p.profiling = enable != 0;
    return IFGF_OK;
}

// Folds the recorded event pairs into the per-stage and per-level totals.
static ifgf_status collect_times(ifgf::DevicePlan& p)
{
    hipError_t e = hipStreamSynchronize(p.last_stream);
    if (e == hipSuccess && p.side) e = hipStreamSynchronize(p.side);
    if (e != hipSuccess) return hip_fail(e, "stage timing");
    for (const auto& q : p.pending) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, p.events[q.e0], p.events[q.e1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        p.stage_ms[q.stage] += t;
        p.stage_launches[q.stage] += 1;
        p.level_ms[q.stage][q.level] += t;
        p.level_launches[q.stage][q.level] += 1;
    }
    p.pending.clear();
    p.next_event = 0;
    return IFGF_OK;
}

ifgf_status ifgf_plan_stage_times(ifgf_plan_t plan, double* ms, int64_t* launches)
{
    if (!plan || !ms || !launches) return fail(IFGF_E_INVALID_ARG, "NULL argument");
    ifgf::DevicePlan& p = plan->p;
    if (p.host_only) return fail(IFGF_E_UNSUPPORTED, "plan was created with host_only");
    DeviceGuard g(p.device);
    ifgf_status s = collect_times(p);
    if (s != IFGF_OK) return s;
    for (int i = 0; i < IFGF_NUM_STAGES; ++i) {
        ms[i] = p.stage_ms[i];
        launches[i] = p.stage_launches[i];
    }
    return IFGF_OK;
}

ifgf_status ifgf_plan_level_times(ifgf_plan_t plan, int32_t stage, double* ms, int64_t* launches)
{
    if (!plan || !ms || !launches) return fail(IFGF_E_INVALID_ARG, "NULL argument");
    if (stage < 0 || stage >= IFGF_NUM_STAGES) return fail(IFGF_E_INVALID_ARG, "unknown stage");
    ifgf::DevicePlan& p = plan->p;
    if (p.host_only) return fail(IFGF_E_UNSUPPORTED, "plan was created with host_only");
    DeviceGuard g(p.device);
    ifgf_status s = collect_times(p);
    if (s != IFGF_OK) return s;
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) {
        ms[d] = p.level_ms[stage][d];
        launches[d] = p.level_launches[stage][d];
    }
    return IFGF_OK;
}

ifgf_status ifgf_plan_destroy(ifgf_plan_t plan)
{
    if (!plan) return IFGF_OK;
    release(plan->p);
    delete plan;
    return IFGF_OK;
}

const char* ifgf_status_string(ifgf_status s)
{
    switch (s) {
    case IFGF_OK: return "IFGF_OK";
    case IFGF_E_INVALID_ARG: return "IFGF_E_INVALID_ARG";
    case IFGF_E_OUT_OF_MEMORY: return "IFGF_E_OUT_OF_MEMORY";
    case IFGF_E_HIP: return "IFGF_E_HIP";
    case IFGF_E_UNSUPPORTED: return "IFGF_E_UNSUPPORTED";
    case IFGF_E_INTERNAL: return "IFGF_E_INTERNAL";
    }
    return "unknown ifgf_status";
}

const char* ifgf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
