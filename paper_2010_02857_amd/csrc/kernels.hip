// HIP kernels of the IFGF operator for gfx950 (Algorithm 1, Sec. 3.3.3).
//
// Every kernel gathers: each output element (a target, or an interpolation
// point of a parent cone) is owned by one thread, which loops over the
// sources that reach it.  No output is written by two threads, so results
// are deterministic and no atomics are needed.  Points are in Morton order,
// so the threads of a wavefront share boxes, cousin lists and cone data.
//
// Precision: T = double gives the FP64 path; T = float the mixed path, in
// which distances, the phase k r and its reduction modulo 2 pi, box centres
// and the cone map (s, theta, phi) stay FP64 while kernel values,
// interpolation weights and accumulation are FP32.
#include "ifgf_internal.hpp"

#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <type_traits>

namespace ifgf {
namespace {

constexpr double k2Pi = 2.0 * kPi;
constexpr double kInv2Pi = 1.0 / (2.0 * kPi);
constexpr double kInv4Pi = 1.0 / (4.0 * kPi);
constexpr int kBlock = 256;

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

// e^{i ph}: FP64 sincos, or for float an FP64 reduction of ph to [-pi, pi]
// followed by FP32 sincos.
template <typename T>
__device__ inline void expi(double ph, T& c, T& s);
// A zero phase (every phase of the Laplace kernel, k = 0) skips the sine
// and cosine: e^0 = 1 exactly, as they would return.
template <>
__device__ inline void expi<double>(double ph, double& c, double& s)
{
    if (ph == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    sincos(ph, &s, &c);
}
template <>
__device__ inline void expi<float>(double ph, float& c, float& s)
{
    if (ph == 0.0) {
        c = 1.0f;
        s = 0.0f;
        return;
    }
    double q = rint(ph * kInv2Pi);
    float red = (float)(ph - q * k2Pi);
    sincosf(red, &s, &c);
}

// The dispatcher hands workgroups to the eight XCDs in turn (workgroup b to
// XCD b mod 8), and each XCD has its own L2.  Neighbouring work items read
// the same cone values, so the workgroup index is renumbered to give each XCD
// one contiguous range of the grid: XCD x takes indices
// [x per + min(x, rem), ...) in dispatch order.  A bijection of [0, nb).
__device__ inline int xcd_block(int b, int nb)
{
    const int x = b & 7, l = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return x * per + (x < rem ? x : rem) + l;
}

// Orders the LDS accesses of one wavefront (which the LDS executes in issue
// order) without waiting for outstanding global loads, so prefetches stay in
// flight across it.
__device__ inline void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Parent slot visited at position i of a child-to-parent launch: with
// ORDERED the box tiles' order (blocks of boxes, one parent cone after the
// other), so that neighbouring work shares frames in cache; else slot order
// (box-major), so that it shares child cones.
template <bool ORDERED>
__device__ inline int slot_at(const LevelDev& Lc, int i)
{
    if constexpr (ORDERED) return Lc.slot_order[i];
    return i;
}

// Lagrange basis of the N first-kind Chebyshev nodes at t:
// L_k(t) = prod_{j != k} (t - t_j) / (t_k - t_j).  Interpolating the node
// values with it gives the same polynomial as the Chebyshev expansion whose
// coefficients the discrete transform would produce.
template <typename T, int N>
__device__ inline void lagrange(double t, const ChebNodes& cn, T* L)
{
    T tt = (T)t;
    T d[N], suf[N];
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = tt - (T)cn.t[k];
    suf[N - 1] = (T)1;
#pragma unroll
    for (int k = N - 2; k >= 0; --k) suf[k] = suf[k + 1] * d[k + 1];
    T pre = (T)1;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        L[k] = pre * suf[k] * (T)cn.inv[k];
        pre *= d[k];
    }
}

// Basis and its derivative d/dt.
template <typename T, int N>
__device__ inline void lagrange_d(double t, const ChebNodes& cn, T* L, T* dL)
{
    T tt = (T)t;
    T d[N];
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = tt - (T)cn.t[k];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        T p = (T)1, dp = (T)0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j == k) continue;
            dp = dp * d[j] + p;
            p *= d[j];
        }
        L[k] = p * (T)cn.inv[k];
        dL[k] = dp * (T)cn.inv[k];
    }
}


// sum_{a,b,c} F[a][b][c][r] Ls[a] Lt[b] Lp[c] for the RB right-hand sides,
// contracted one direction at a time (phi, then theta, then s), which needs
// no products of the three weights.  With one right-hand side everything is
// unrolled; with several, the (a, b) loop is kept rolled so that the
// compiler cannot hoist all P * RB loads at once and spill.
template <typename T, int PS, int PA, int RB>
__device__ inline void interp(const cpx<T>* __restrict__ F, const T* Ls, const T* Lt, const T* Lp, cpx<T>* v)
{
#pragma unroll
    for (int r = 0; r < RB; ++r) v[r].x = v[r].y = (T)0;
    if constexpr (RB == 1) {
#pragma unroll
        for (int a = 0; a < PS; ++a) {
            T wx = (T)0, wy = (T)0;
#pragma unroll
            for (int b = 0; b < PA; ++b) {
                T ux = (T)0, uy = (T)0;
#pragma unroll
                for (int c = 0; c < PA; ++c) {
                    cpx<T> q = F[(a * PA + b) * PA + c];
                    ux += Lp[c] * q.x;
                    uy += Lp[c] * q.y;
                }
                wx += Lt[b] * ux;
                wy += Lt[b] * uy;
            }
            v[0].x += Ls[a] * wx;
            v[0].y += Ls[a] * wy;
        }
    } else {
        cpx<T> w[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) w[r].x = w[r].y = (T)0;
#pragma unroll 1
        for (int ab = 0; ab < PS * PA; ++ab) {
            const int a = ab / PA, b = ab - a * PA;
            T la = Ls[0], lb = Lt[0];
#pragma unroll
            for (int i = 1; i < PS; ++i) la = a == i ? Ls[i] : la;
#pragma unroll
            for (int i = 1; i < PA; ++i) lb = b == i ? Lt[i] : lb;
            const cpx<T>* f = F + ab * PA * RB;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                T ux = (T)0, uy = (T)0;
#pragma unroll
                for (int c = 0; c < PA; ++c) {
                    cpx<T> q = f[c * RB + r];
                    ux += Lp[c] * q.x;
                    uy += Lp[c] * q.y;
                }
                w[r].x += lb * ux;
                w[r].y += lb * uy;
            }
            if (b == PA - 1) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    v[r].x += la * w[r].x;
                    v[r].y += la * w[r].y;
                    w[r].x = w[r].y = (T)0;
                }
            }
        }
    }
}

// ------------------------------------- node counts known only at run time
//
// Kernels instantiated with PS = PA = 0 serve plans whose node counts were
// not compiled in: P_s = kc.ps and P_ang = kc.pa (each 1..kMaxNodes) are read
// at run time, the basis arrays are kMaxNodes long, and every loop runs to
// kMaxNodes with a guard so that the arrays stay in registers.

// Lagrange basis through the first n of the nodes cn at t (zeros beyond n).
template <typename T>
__device__ inline void lagrange_any(double t, const ChebNodes& cn, int n, T* L)
{
    const T tt = (T)t;
    T d[kMaxNodes], suf[kMaxNodes];
#pragma unroll
    for (int k = 0; k < kMaxNodes; ++k) d[k] = tt - (T)cn.t[k];
    suf[kMaxNodes - 1] = (T)1;
#pragma unroll
    for (int k = kMaxNodes - 2; k >= 0; --k) suf[k] = k + 1 < n ? suf[k + 1] * d[k + 1] : (T)1;
    T pre = (T)1;
#pragma unroll
    for (int k = 0; k < kMaxNodes; ++k) {
        L[k] = k < n ? pre * suf[k] * (T)cn.inv[k] : (T)0;
        pre *= d[k];
    }
}

// The basis and its derivative d/dt (zeros beyond n).
template <typename T>
__device__ inline void lagrange_d_any(double t, const ChebNodes& cn, int n, T* L, T* dL)
{
    const T tt = (T)t;
    T d[kMaxNodes];
#pragma unroll
    for (int k = 0; k < kMaxNodes; ++k) d[k] = tt - (T)cn.t[k];
#pragma unroll
    for (int k = 0; k < kMaxNodes; ++k) {
        T p = (T)1, dp = (T)0;
#pragma unroll
        for (int j = 0; j < kMaxNodes; ++j) {
            if (j == k || j >= n) continue;
            dp = dp * d[j] + p;
            p *= d[j];
        }
        L[k] = k < n ? p * (T)cn.inv[k] : (T)0;
        dL[k] = k < n ? dp * (T)cn.inv[k] : (T)0;
    }
}

// Element i < kMaxNodes of a register array, by a chain of selects.
template <typename T>
__device__ inline T sel_any(const T* a, int i)
{
    T v = a[0];
#pragma unroll
    for (int k = 1; k < kMaxNodes; ++k) v = i == k ? a[k] : v;
    return v;
}

// interp for run-time node counts ps x pa x pa: phi contracted first (in
// registers), then theta and s.
template <typename T, int RB>
__device__ inline void interp_any(const cpx<T>* __restrict__ F, const T* Ls, const T* Lt, const T* Lp, int ps,
                                  int pa, cpx<T>* v)
{
#pragma unroll
    for (int r = 0; r < RB; ++r) v[r].x = v[r].y = (T)0;
    for (int a = 0; a < ps; ++a) {
        const T la = sel_any(Ls, a);
        cpx<T> w[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) w[r].x = w[r].y = (T)0;
        for (int b = 0; b < pa; ++b) {
            const T lb = sel_any(Lt, b);
            const cpx<T>* f = F + (size_t)(a * pa + b) * pa * RB;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                T ux = (T)0, uy = (T)0;
#pragma unroll
                for (int c = 0; c < kMaxNodes; ++c) {
                    if (c < pa) {
                        const cpx<T> q = f[c * RB + r];
                        ux += Lp[c] * q.x;
                        uy += Lp[c] * q.y;
                    }
                }
                w[r].x += lb * ux;
                w[r].y += lb * uy;
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            v[r].x += la * w[r].x;
            v[r].y += la * w[r].y;
        }
    }
}

// Dispatch between the compiled node counts (N > 0) and run-time ones (N = 0).
template <int N>
constexpr int basis_len()
{
    return N > 0 ? N : kMaxNodes;
}
template <typename T, int N>
__device__ inline void basis(double t, const ChebNodes& cn, int n, T* L)
{
    if constexpr (N > 0) lagrange<T, N>(t, cn, L);
    else lagrange_any<T>(t, cn, n, L);
}
template <typename T, int N>
__device__ inline void basis_d(double t, const ChebNodes& cn, int n, T* L, T* dL)
{
    if constexpr (N > 0) lagrange_d<T, N>(t, cn, L, dL);
    else lagrange_d_any<T>(t, cn, n, L, dL);
}
template <typename T, int PS, int PA, int RB>
__device__ inline void interp_n(const cpx<T>* __restrict__ F, const T* Ls, const T* Lt, const T* Lp,
                                const KernelConsts& kc, cpx<T>* v)
{
    if constexpr (PS > 0) interp<T, PS, PA, RB>(F, Ls, Lt, Lp, v);
    else interp_any<T, RB>(F, Ls, Lt, Lp, kc.ps, kc.pa, v);
}

// ------------------------------------------------------------------ kernels

// A window [w0, w0 + wn) of the plan's point indices (input order): all
// points, or with distinct targets the sources [0, n_src) or the targets
// [n_src, n_src + n_tgt).
struct Window {
    int w0, wn;
};

// values on a window, [nrhs][wn] (input order) -> [n][RB] (Morton order),
// zero outside the window and for right-hand sides beyond nrhs.
template <typename T, int RB>
__global__ void __launch_bounds__(kBlock) k_permute_in(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                                       const int32_t* __restrict__ perm, int n, Window w, int nrhs,
                                                       int r0)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int src = perm[i] - w.w0;
    const bool inside = src >= 0 && src < w.wn;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        int rr = r0 + r;
        cpx<T> v;
        v.x = v.y = (T)0;
        if (rr < nrhs && inside) v = in[(size_t)rr * w.wn + src];
        out[(size_t)i * RB + r] = v;
    }
}

// [n][RB] (Morton order) -> out [nrhs][wn], the window's points (input order).
template <typename T, int RB>
__global__ void __launch_bounds__(kBlock) k_permute_out(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                                        const int32_t* __restrict__ iperm, Window w, int nrhs, int r0)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= w.wn) return;
    int i = iperm[w.w0 + j];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        int rr = r0 + r;
        if (rr < nrhs) out[(size_t)rr * w.wn + j] = in[(size_t)i * RB + r];
    }
}

// The sources summed directly at the targets of level-D box b, as Morton
// point ranges e in [near_first, near_end): the box's neighbours, or with an
// adaptive octree the leaves (of any level) whose neighbourhood holds it.
__device__ inline int near_first(const LevelDev& L, int b) { return L.near_start ? L.near_start[b] : L.nbr_start[b]; }
__device__ inline int near_end(const LevelDev& L, int b) { return L.near_start ? L.near_start[b + 1] : L.nbr_start[b + 1]; }
__device__ inline void near_range(const LevelDev& L, int e, int& lo, int& hi)
{
    if (L.near_start) {
        lo = L.near_lo[e];
        hi = L.near_hi[e];
    } else {
        const int q = L.nbr[e];
        lo = L.box_start[q];
        hi = L.box_start[q + 1];
    }
}

// Near field (Algorithm 1, direct evaluations onto the neighbourhood U B):
// I(x_i) = sum over the neighbour boxes of x_i's leaf box of a_j G(x_i, x_j),
// j != i.  Writes (initialises) the output.
template <typename T, int RB>
__global__ void __launch_bounds__(kBlock) k_nearfield(KernelConsts kc, LevelDev L, const double* __restrict__ pts,
                                                      const cpx<T>* __restrict__ dens, cpx<T>* __restrict__ out)
{
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int b = L.pt_box[i];
    const double x0 = pts[3 * i], x1 = pts[3 * i + 1], x2 = pts[3 * i + 2];
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    const int e1 = near_end(L, b);
    for (int e = near_first(L, b); e < e1; ++e) {
        int lo, hi;
        near_range(L, e, lo, hi);
        for (int j = lo; j < hi; ++j) {
            if (j == i) continue;
            double dx = x0 - pts[3 * j], dy = x1 - pts[3 * j + 1], dz = x2 - pts[3 * j + 2];
            double rr = sqrt(dx * dx + dy * dy + dz * dz);
            T c, s;
            expi<T>(kc.kappa * rr, c, s);
            T inv = (T)(kInv4Pi / rr);
            T gr = c * inv, gi = s * inv;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                cpx<T> a = dens[(size_t)j * RB + r];
                acc[r].x += a.x * gr - a.y * gi;
                acc[r].y += a.x * gi + a.y * gr;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) out[(size_t)i * RB + r] = acc[r];
}

// Leaf boxes: F_k at every interpolation point of every relevant cone of a
// leaf box (eq. I_k): F(x) = sum_{m in B_k} a_m |x - c| / |x - x_m| e^{i k (|x - x_m| - |x - c|)},
// the difference of radii formed as (|w|^2 - 2 y.w) / (|y - w| + |y|) with
// y = x - c, w = x_m - c.  Every slot of level D (list null), or the slots
// list[0..nlist) of the leaf boxes of a coarser level (adaptive octree).
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_leaf_nodes(KernelConsts kc, LevelDev L, const double* __restrict__ pts,
                                                       const cpx<T>* __restrict__ dens, cpx<T>* __restrict__ F,
                                                       const int32_t* __restrict__ list, int nlist)
{
    const int ps = PS > 0 ? PS : kc.ps, pa = PA > 0 ? PA : kc.pa;
    const int P = ps * pa * pa;
    size_t gid = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    int slot = (int)(gid / P);
    int nu = (int)(gid - (size_t)slot * P);
    if (slot >= (list ? nlist : L.nslots)) return;
    if (list) slot = list[slot];
    const int b = L.slot_box[slot];
    const int cone = L.slot_cone[slot];
    const int cell = cone / L.ns, is = cone - cell * L.ns;
    const int a = nu / (pa * pa), bc = nu - a * pa * pa;
    const double rr = L.node_r[is * ps + a];
    const double* dir = &L.node_dir[((size_t)cell * pa * pa + bc) * 3];
    const double y0 = rr * dir[0], y1 = rr * dir[1], y2 = rr * dir[2];
    const double ry = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    const double c0 = L.box_ctr[3 * b], c1 = L.box_ctr[3 * b + 1], c2 = L.box_ctr[3 * b + 2];
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int j = L.box_start[b]; j < L.box_start[b + 1]; ++j) {
        double w0 = pts[3 * j] - c0, w1 = pts[3 * j + 1] - c1, w2 = pts[3 * j + 2] - c2;
        double e0 = y0 - w0, e1 = y1 - w1, e2 = y2 - w2;
        double rxy = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        double num = (w0 * w0 + w1 * w1 + w2 * w2) - 2.0 * (y0 * w0 + y1 * w1 + y2 * w2);
        double diff = num / (rxy + ry);
        T c, s;
        expi<T>(kc.kappa * diff, c, s);
        T mag = (T)(ry / rxy);
        T gr = mag * c, gi = mag * s;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            cpx<T> q = dens[(size_t)j * RB + r];
            acc[r].x += q.x * gr - q.y * gi;
            acc[r].y += q.x * gi + q.y * gr;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) F[((size_t)slot * P + nu) * RB + r] = acc[r];
}

// Interpolation at cousin targets, level d (Algorithm 1, first inner loop):
// for target x and every cousin box k of x's box,
//   I(x) += G(x, x_k) P_{k, gamma(x)}(s, theta, phi).
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_eval(KernelConsts kc, LevelDev L, const double* __restrict__ pts,
                                                        const cpx<T>* __restrict__ F, cpx<T>* __restrict__ out)
{
    const int P = PS > 0 ? PS * PA * PA : kc.ps * kc.pa * kc.pa;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int t = L.pt_box[i];
    const double x0 = pts[3 * i], x1 = pts[3 * i + 1], x2 = pts[3 * i + 2];
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int ci = L.cou_start[t]; ci < L.cou_start[t + 1]; ++ci) {
        const int k = L.cou[ci];
        ConeLoc cl;
        cone_locate(x0 - L.box_ctr[3 * k], x1 - L.box_ctr[3 * k + 1], x2 - L.box_ctr[3 * k + 2], L.h, L.ds, L.dang,
                    L.ns, L.nc, cl);
        const int slot = lookup(L, k, cl.cell, cl.is);
        if (slot < 0) {
            atomicAdd(kc.miss, 1ull);
            continue;
        }
        T Ls[basis_len<PS>()], Lt[basis_len<PA>()], Lp[basis_len<PA>()];
        basis<T, PS>(cl.ts, kc.cs, kc.ps, Ls);
        basis<T, PA>(cl.tt, kc.ca, kc.pa, Lt);
        basis<T, PA>(cl.tp, kc.ca, kc.pa, Lp);
        cpx<T> v[RB];
        interp_n<T, PS, PA, RB>(F + (size_t)slot * P * RB, Ls, Lt, Lp, kc, v);
        T c, s;
        expi<T>(kc.kappa * cl.r, c, s);
        T inv = (T)(kInv4Pi / cl.r);
        T gr = c * inv, gi = s * inv;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            acc[r].x += v[r].x * gr - v[r].y * gi;
            acc[r].y += v[r].x * gi + v[r].y * gr;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        cpx<T> o = out[(size_t)i * RB + r];
        o.x += acc[r].x;
        o.y += acc[r].y;
        out[(size_t)i * RB + r] = o;
    }
}

// Interpolation at cousin targets through the tabulated pairs: the slot,
// local coordinates and centred factor of (target, cousin box) were computed
// with the plan, so no FP64 geometry is left.  Entries of one target box are
// stored cousin-major, so the targets of a box read consecutive entries.
// The centred factor is conjugated for the adjoint (kc.adj).
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_eval_pairs(KernelConsts kc, LevelDev L,
                                                              const cpx<T>* __restrict__ F, cpx<T>* __restrict__ out)
{
    constexpr int P = PS * PA * PA;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int tb = L.pt_box[i];
    const int b0 = L.box_start[tb];
    const long long nT = L.box_start[tb + 1] - b0;
    const int tl = i - b0;
    const long long base = L.pair_base[tb];
    const int nc = L.cou_start[tb + 1] - L.cou_start[tb];
    const long long np = L.npairs_cou;
    const T* pt = (const T*)L.pr_t;
    const T* pg = (const T*)L.pr_g;
    const T conj_sign = kc.adj ? (T)-1 : (T)1;
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int c = 0; c < nc; ++c) {
        const long long e = base + c * nT + tl;
        const int slot = L.pr_slot[e];
        if (slot < 0) {
            atomicAdd(kc.miss, 1ull);
            continue;
        }
        T Ls[PS], Lt[PA], Lp[PA];
        lagrange<T, PS>((double)pt[e], kc.cs, Ls);
        lagrange<T, PA>((double)pt[np + e], kc.ca, Lt);
        lagrange<T, PA>((double)pt[2 * np + e], kc.ca, Lp);
        cpx<T> v[RB];
        interp<T, PS, PA, RB>(F + (size_t)slot * P * RB, Ls, Lt, Lp, v);
        const T gr = pg[e], gi = conj_sign * pg[np + e];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            acc[r].x += v[r].x * gr - v[r].y * gi;
            acc[r].y += v[r].x * gi + v[r].y * gr;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        cpx<T> o = out[(size_t)i * RB + r];
        o.x += acc[r].x;
        o.y += acc[r].y;
        out[(size_t)i * RB + r] = o;
    }
}

// Two-phase interpolation at cousin targets (one right-hand side), through
// the tabulated pairs.  Phase 1 takes the pairs in cone-slot order, from a
// copy of the pair table in that order, so the threads of a wavefront read
// consecutive pair data and one or two cones, served from cache; each pair's
// interpolated value times its centred factor is stored at the pair's place
// in target order.  Phase 2 adds, for every target, the values of its
// pairs in cousin order.  No atomics: the sums have a fixed order.
template <typename T, int PS, int PA>
__global__ void __launch_bounds__(kBlock) k_cousin_pairs_values(KernelConsts kc, LevelDev L,
                                                                const cpx<T>* __restrict__ F,
                                                                cpx<T>* __restrict__ pval)
{
    // kPairQuad consecutive entries share a cone: one thread interpolates them
    // together, reading each cone value once (phi, then theta, then s)
    constexpr int P = PS * PA * PA;
    constexpr int QR = kPairQuad;
    const long long i0 = ((long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) * QR;
    const long long no = L.npairs_ord;
    if (i0 >= no) return;
    const int slot = L.pro_slot[i0];
    const T* pt = (const T*)L.pro_t;
    const T* pg = (const T*)L.pro_g;
    T Ls[QR][PS], Lt[QR][PA], Lq[QR][PA];
#pragma unroll
    for (int r = 0; r < QR; ++r) {
        lagrange<T, PS>((double)pt[i0 + r], kc.cs, Ls[r]);
        lagrange<T, PA>((double)pt[no + i0 + r], kc.ca, Lt[r]);
        lagrange<T, PA>((double)pt[2 * no + i0 + r], kc.ca, Lq[r]);
    }
    const cpx<T>* Fs = F + (size_t)slot * P;
    cpx<T> U[QR][PS];
#pragma unroll
    for (int r = 0; r < QR; ++r)
#pragma unroll
        for (int a = 0; a < PS; ++a) U[r][a] = cpx<T>{(T)0, (T)0};
    // one phi-row of the cone per step; the theta loop stays rolled (its
    // weights shift through registers) so that the loads are issued row by
    // row instead of all at once
#pragma unroll
    for (int a = 0; a < PS; ++a) {
        T lt[QR][PA];
#pragma unroll
        for (int r = 0; r < QR; ++r)
#pragma unroll
            for (int c = 0; c < PA; ++c) lt[r][c] = Lt[r][c];
        const cpx<T>* Fa = Fs + a * PA * PA;
#pragma unroll 1
        for (int b = 0; b < PA; ++b) {
            cpx<T> fv[PA];
#pragma unroll
            for (int c = 0; c < PA; ++c) fv[c] = Fa[b * PA + c];
#pragma unroll
            for (int r = 0; r < QR; ++r) {
                T sr = (T)0, si = (T)0;
#pragma unroll
                for (int c = 0; c < PA; ++c) {
                    sr += fv[c].x * Lq[r][c];
                    si += fv[c].y * Lq[r][c];
                }
                U[r][a].x += sr * lt[r][0];
                U[r][a].y += si * lt[r][0];
#pragma unroll
                for (int c = 0; c + 1 < PA; ++c) lt[r][c] = lt[r][c + 1];
            }
        }
    }
    const T sg = kc.adj ? (T)-1 : (T)1;
#pragma unroll
    for (int r = 0; r < QR; ++r) {
        const int e = L.pr_order[i0 + r];
        if (e < 0) continue;
        T vr = (T)0, vi = (T)0;
#pragma unroll
        for (int a = 0; a < PS; ++a) {
            vr += U[r][a].x * Ls[r][a];
            vi += U[r][a].y * Ls[r][a];
        }
        const T gr = pg[i0 + r], gi = sg * pg[no + i0 + r];
        pval[e] = cpx<T>{vr * gr - vi * gi, vr * gi + vi * gr};
    }
}

template <typename T, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_pairs_sum(KernelConsts kc, LevelDev L,
                                                             const cpx<T>* __restrict__ pval,
                                                             cpx<T>* __restrict__ out)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int tb = L.pt_box[i];
    const int b0 = L.box_start[tb];
    const long long nT = L.box_start[tb + 1] - b0;
    const long long base = L.pair_base[tb] + (i - b0);
    const int nc = L.cou_start[tb + 1] - L.cou_start[tb];
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int c = 0; c < nc; ++c) {
        const long long e = base + c * nT;
        if (L.pr_slot[e] < 0) {
            atomicAdd(kc.miss, 1ull);
            continue;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cpx<T> v = pval[e * RB + r];
            acc[r].x += v.x;
            acc[r].y += v.y;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        cpx<T> o = out[(size_t)i * RB + r];
        o.x += acc[r].x;
        o.y += acc[r].y;
        out[(size_t)i * RB + r] = o;
    }
}


// Largest b in [0, n) with start[b] <= x (start ascending, start[0] <= x).
__device__ inline int box_of_pair(const long long* start, int n, long long x)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Cousin-target interpolation in two phases on levels without tabulated
// pairs.  Phase 1: one thread per (target box T, cousin c, target t) pair,
// in the order of the pair tables (entry pair_off[T] + c n_T + t), computes
// the target's cone of the cousin box, the interpolant there and the centred
// factor G(x_t, x_c), and stores the product.  Neighbouring threads share T
// and c, and mostly one cone, so their reads of the cone values coalesce
// (the one-kernel form reads each pair's 75 x RB values in its own thread).
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_pairs_geo(KernelConsts kc, LevelDev L,
                                                             const double* __restrict__ pts,
                                                             const long long* __restrict__ pair_off, long long np,
                                                             const cpx<T>* __restrict__ F,
                                                             cpx<T>* __restrict__ pval)
{
    constexpr int P = PS * PA * PA;
    const long long e = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (e >= np) return;
    const int tb = box_of_pair(pair_off, L.nbox, e);
    const int b0 = L.box_start[tb];
    const int nT = L.box_start[tb + 1] - b0;
    const long long rel = e - pair_off[tb];
    const int ci = (int)(rel / nT), t = (int)(rel - (long long)ci * nT);
    const int k = L.cou[L.cou_start[tb] + ci];
    const int i = b0 + t;
    ConeLoc cl;
    cone_locate(pts[3 * i] - L.box_ctr[3 * k], pts[3 * i + 1] - L.box_ctr[3 * k + 1], pts[3 * i + 2] - L.box_ctr[3 * k + 2],
                L.h, L.ds, L.dang, L.ns, L.nc, cl);
    const int slot = lookup(L, k, cl.cell, cl.is);
    cpx<T> v[RB];
    if (slot < 0) {
        atomicAdd(kc.miss, 1ull);
#pragma unroll
        for (int r = 0; r < RB; ++r) v[r].x = v[r].y = (T)0;
    } else {
        T Ls[PS], Lt[PA], Lp[PA];
        lagrange<T, PS>(cl.ts, kc.cs, Ls);
        lagrange<T, PA>(cl.tt, kc.ca, Lt);
        lagrange<T, PA>(cl.tp, kc.ca, Lp);
        interp<T, PS, PA, RB>(F + (size_t)slot * P * RB, Ls, Lt, Lp, v);
        T c, s;
        expi<T>(kc.kappa * cl.r, c, s);
        const T inv = (T)(kInv4Pi / cl.r);
        const T gr = c * inv, gi = s * inv;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const T x = v[r].x * gr - v[r].y * gi, y = v[r].x * gi + v[r].y * gr;
            v[r].x = x;
            v[r].y = y;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) pval[e * RB + r] = v[r];
}

// The same phase 1 through a level's pair table (slot, local coordinates and
// centred factor tabulated in target order): one thread per pair, so that
// neighbouring threads read the same cone values (the one-kernel form,
// k_cousin_eval_pairs, walks one target's cousins per thread).  Phase 2 is
// k_cousin_pairs_sum.
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_pairs_tab(KernelConsts kc, LevelDev L,
                                                             const cpx<T>* __restrict__ F,
                                                             cpx<T>* __restrict__ pval)
{
    constexpr int P = PS * PA * PA;
    const long long e = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const long long np = L.npairs_cou;
    if (e >= np) return;
    const int slot = L.pr_slot[e];
    cpx<T> v[RB];
    if (slot < 0) {
        // counted by the sum
#pragma unroll
        for (int r = 0; r < RB; ++r) v[r].x = v[r].y = (T)0;
    } else {
        const T* pt = (const T*)L.pr_t;
        const T* pg = (const T*)L.pr_g;
        T Ls[PS], Lt[PA], Lp[PA];
        lagrange<T, PS>((double)pt[e], kc.cs, Ls);
        lagrange<T, PA>((double)pt[np + e], kc.ca, Lt);
        lagrange<T, PA>((double)pt[2 * np + e], kc.ca, Lp);
        interp<T, PS, PA, RB>(F + (size_t)slot * P * RB, Ls, Lt, Lp, v);
        const T gr = pg[e], gi = (kc.adj ? (T)-1 : (T)1) * pg[np + e];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const T x = v[r].x * gr - v[r].y * gi, y = v[r].x * gi + v[r].y * gr;
            v[r].x = x;
            v[r].y = y;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) pval[e * RB + r] = v[r];
}

// Phase 2: every target adds its pairs' values in cousin order (one thread
// per target, no atomics, so the result does not depend on scheduling).
template <typename T, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_pairs_sum_geo(KernelConsts kc, LevelDev L,
                                                                 const long long* __restrict__ pair_off,
                                                                 const cpx<T>* __restrict__ pval,
                                                                 cpx<T>* __restrict__ out)
{
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int tb = L.pt_box[i];
    const int b0 = L.box_start[tb];
    const long long nT = L.box_start[tb + 1] - b0;
    const long long base = pair_off[tb] + (i - b0);
    const int nc = L.cou_start[tb + 1] - L.cou_start[tb];
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int c = 0; c < nc; ++c) {
        const long long e = base + c * nT;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const cpx<T> v = pval[e * RB + r];
            acc[r].x += v.x;
            acc[r].y += v.y;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        cpx<T> o = out[(size_t)i * RB + r];
        o.x += acc[r].x;
        o.y += acc[r].y;
        out[(size_t)i * RB + r] = o;
    }
}

// Child-to-parent interpolation, children at level d (Algorithm 1, second
// inner loop): for every interpolation point x of every relevant cone of a
// level-(d-1) box j,
//   F_j(x) = sum_{children k} P_{k, gamma(x)}(.) G(x, x_k) / G(x, x_j),
// with G(x, x_k) / G(x, x_j) = |y| / |y - o| e^{i k (|y - o| - |y|)},
// y = x - x_j, o = x_k - x_j, and |y - o| - |y| = (|o|^2 - 2 y.o) / (|y - o| + |y|).
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_child_to_parent(KernelConsts kc, LevelDev Lc, LevelDev Lp,
                                                            const cpx<T>* __restrict__ Fc, cpx<T>* __restrict__ Fp)
{
    const int ps = PS > 0 ? PS : kc.ps, pa = PA > 0 ? PA : kc.pa;
    const int P = ps * pa * pa;
    size_t gid = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    int pslot = (int)(gid / P);
    int nu = (int)(gid - (size_t)pslot * P);
    if (pslot >= Lp.nslots) return;
    const int j = Lp.slot_box[pslot];
    const int pcone = Lp.slot_cone[pslot];
    const int pcell = pcone / Lp.ns, pis = pcone - pcell * Lp.ns;
    const int a = nu / (pa * pa), bc = nu - a * pa * pa;
    const double rr = Lp.node_r[pis * ps + a];
    const double* dir = &Lp.node_dir[((size_t)pcell * pa * pa + bc) * 3];
    const double y0 = rr * dir[0], y1 = rr * dir[1], y2 = rr * dir[2];
    const double ry = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    const double half = 0.5 * Lc.H;
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int k = Lp.chl_start[j]; k < Lp.chl_start[j + 1]; ++k) {
        const int oct = Lc.box_oct[k];
        if (Lc.child_of[(size_t)j * 8 + oct] != k) continue;   // below a leaf (adaptive octree)
        double o[3] = {(oct & 1) ? half : -half, (oct & 2) ? half : -half, (oct & 4) ? half : -half};
        double v[3];
        node_minus(rr, dir, o, v);
        ConeLoc cl;
        cone_locate(v[0], v[1], v[2], Lc.h, Lc.ds, Lc.dang, Lc.ns, Lc.nc, cl);
        const int slot = lookup(Lc, k, cl.cell, cl.is);
        if (slot < 0) {
            atomicAdd(kc.miss, 1ull);
            continue;
        }
        T Ls[basis_len<PS>()], Lt[basis_len<PA>()], Lpp[basis_len<PA>()];
        basis<T, PS>(cl.ts, kc.cs, kc.ps, Ls);
        basis<T, PA>(cl.tt, kc.ca, kc.pa, Lt);
        basis<T, PA>(cl.tp, kc.ca, kc.pa, Lpp);
        cpx<T> val[RB];
        interp_n<T, PS, PA, RB>(Fc + (size_t)slot * P * RB, Ls, Lt, Lpp, kc, val);
        double num = (o[0] * o[0] + o[1] * o[1] + o[2] * o[2]) - 2.0 * (y0 * o[0] + y1 * o[1] + y2 * o[2]);
        double diff = num / (cl.r + ry);
        T c, s;
        expi<T>(kc.kappa * diff, c, s);
        T mag = (T)(ry / cl.r);
        T gr = mag * c, gi = mag * s;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            acc[r].x += val[r].x * gr - val[r].y * gi;
            acc[r].y += val[r].x * gi + val[r].y * gr;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) Fp[((size_t)pslot * P + nu) * RB + r] = acc[r];
}

// Child-to-parent interpolation through tabulated frames: the child cone,
// local coordinates and re-centring ratio of interpolation point nu of the
// parent cone of slot `pslot` seen from the child in octant o are read from
// the frame of (parent cone, o); only the child's slot is looked up.  For
// the adjoint (kc.adj) the tabulated ratio is conjugated.
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_child_to_parent_frames(KernelConsts kc, LevelDev Lc, LevelDev Lp,
                                                                   const cpx<T>* __restrict__ Fc,
                                                                   cpx<T>* __restrict__ Fp)
{
    constexpr int P = PS * PA * PA;
    size_t gid = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    int pslot = (int)(gid / P);
    int nu = (int)(gid - (size_t)pslot * P);
    if (pslot >= Lp.nslots) return;
    const int j = Lp.slot_box[pslot];
    const T* frt = (const T*)Lc.fr_t;
    const T* frr = (const T*)Lc.fr_ratio;
    const T conj_sign = kc.adj ? (T)-1 : (T)1;
    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int o = 0; o < 8; ++o) {
        const int f = Lc.pframe[(size_t)pslot * 8 + o];
        if (f < 0) continue;
        const int k = Lc.child_of[(size_t)j * 8 + o];
        const size_t e = (size_t)f * P + nu;
        const unsigned key = Lc.fr_key[e];
        const int cell = (int)(key / (unsigned)Lc.ns), is = (int)(key - (unsigned)cell * Lc.ns);
        const int slot = lookup(Lc, k, cell, is);
        if (slot < 0) {
            atomicAdd(kc.miss, 1ull);
            continue;
        }
        T Ls[PS], Lt[PA], Lpp[PA];
        lagrange<T, PS>((double)frt[3 * e], kc.cs, Ls);
        lagrange<T, PA>((double)frt[3 * e + 1], kc.ca, Lt);
        lagrange<T, PA>((double)frt[3 * e + 2], kc.ca, Lpp);
        cpx<T> val[RB];
        interp<T, PS, PA, RB>(Fc + (size_t)slot * P * RB, Ls, Lt, Lpp, val);
        const T gr = frr[2 * e], gi = conj_sign * frr[2 * e + 1];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            acc[r].x += val[r].x * gr - val[r].y * gi;
            acc[r].y += val[r].x * gi + val[r].y * gr;
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) Fp[((size_t)pslot * P + nu) * RB + r] = acc[r];
}

// Child-to-parent interpolation through frames, with the child cones staged
// in LDS.  A block handles S consecutive parent slots.  It first gathers the
// (slot, octant, group) entries of all its frames -- each group is one
// distinct child cone a frame touches, on average 2-3 -- looks up their child
// slots in parallel, copies each cone once from global memory into LDS, and
// then every (slot, interpolation point) thread interpolates from LDS for all
// eight octants.  A block whose cones exceed the LDS capacity GCAP stages
// them in several rounds.  With ORD the slots are visited in the box tiles'
// order (see slot_at), else in slot order (box-major).
template <typename T, int PS, int PA, int RB, int S, int GCAP, bool ORD, int NT>
__global__ void __launch_bounds__(NT) k_child_to_parent_lds(KernelConsts kc, LevelDev Lc, LevelDev Lp,
                                                            const cpx<T>* __restrict__ Fc,
                                                            cpx<T>* __restrict__ Fp)
{
    constexpr int P = PS * PA * PA;
    constexpr int G = kMaxFrameGroups;
    constexpr int MAXE = S * 8 * G;
    static_assert(S * P <= NT, "block too small");
    static_assert(S * 8 <= 64, "the (slot, octant) table must fit one wavefront");
    __shared__ cpx<T> cone[GCAP * P * RB];
    __shared__ int sof[S * 8];        // frame of (slot, octant), -1 none
    __shared__ int soff[S * 8 + 1];   // first entry of (slot, octant)
    __shared__ int staged[MAXE];      // child slot of each entry, -1 missing

    const int tid = threadIdx.x;
    const int slot0 = xcd_block(blockIdx.x, gridDim.x) * S;
    const int s_me = tid / P;
    const int nu = tid - s_me * P;
    const bool active = s_me < S && slot0 + s_me < Lp.nslots;
    const int sp = active ? slot_at<ORD>(Lc, slot0 + s_me) : 0;
    const T* frt = (const T*)Lc.fr_t;
    const T* frr = (const T*)Lc.fr_ratio;
    const T conj_sign = kc.adj ? (T)-1 : (T)1;

    // (slot, octant) frames and an inclusive scan of their group counts
    if (tid < 64) {
        int f = -1, ng = 0;
        if (tid < S * 8) {
            const int qi = slot0 + tid / 8;
            if (qi < Lp.nslots) {
                f = Lc.pframe[(size_t)slot_at<ORD>(Lc, qi) * 8 + (tid & 7)];
                if (f >= 0) ng = Lc.fr_ngrp[f];
            }
        }
        int x = ng;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            int y = __shfl_up(x, dd, 64);
            if (tid >= dd) x += y;
        }
        if (tid < S * 8) {
            sof[tid] = f;
            soff[tid + 1] = x;
        }
        if (tid == 0) soff[0] = 0;
    }
    __syncthreads();
    const int nent = soff[S * 8];
    // child slot of every entry
    for (int i = tid; i < nent; i += NT) {
        int so = 0;
        while (soff[so + 1] <= i) ++so;
        const int f = sof[so];
        const int g = i - soff[so];
        const int q = slot_at<ORD>(Lc, slot0 + so / 8), o = so & 7;
        const int k = Lc.child_of[(size_t)Lp.slot_box[q] * 8 + o];
        const unsigned key = Lc.fr_gkey[(size_t)f * G + g];
        const int cell = (int)(key / (unsigned)Lc.ns), is = (int)(key - (unsigned)cell * Lc.ns);
        staged[i] = lookup(Lc, k, cell, is);
    }
    __syncthreads();

    cpx<T> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r].x = acc[r].y = (T)0;
    for (int base = 0; base < nent; base += GCAP) {
        const int cnt = nent - base < GCAP ? nent - base : GCAP;
        const int total = cnt * P * RB;
        for (int i = tid; i < total; i += NT) {
            const int q = i / (P * RB), off = i - q * (P * RB);
            const int gs = staged[base + q];
            if (gs >= 0) cone[i] = Fc[(size_t)gs * P * RB + off];
        }
        __syncthreads();
        if (active) {
            // the frame data of octant o + 1 is loaded while octant o is computed
            auto frame_of = [&](int o, int& grp, T& ta, T& tb, T& tc, T& ga, T& gb) {
                const int f = sof[s_me * 8 + o];
                const size_t e = (size_t)(f >= 0 ? f : 0) * P + nu;
                grp = Lc.fr_grp[e];
                ta = frt[3 * e];
                tb = frt[3 * e + 1];
                tc = frt[3 * e + 2];
                ga = frr[2 * e];
                gb = frr[2 * e + 1];
            };
            int grp_n;
            T ta_n, tb_n, tc_n, ga_n, gb_n;
            frame_of(0, grp_n, ta_n, tb_n, tc_n, ga_n, gb_n);
            for (int o = 0; o < 8; ++o) {
                const int grp = grp_n;
                const T t0 = ta_n, t1 = tb_n, t2 = tc_n, g0 = ga_n, g1 = gb_n;
                if (o + 1 < 8) frame_of(o + 1, grp_n, ta_n, tb_n, tc_n, ga_n, gb_n);
                const int f = sof[s_me * 8 + o];
                if (f < 0) continue;
                const int ent = soff[s_me * 8 + o] + grp;
                const int pos = ent - base;
                if (pos < 0 || pos >= cnt) continue;
                if (staged[ent] < 0) {
                    atomicAdd(kc.miss, 1ull);
                    continue;
                }
                T Ls[PS], Lt[PA], Lpp[PA];
                lagrange<T, PS>((double)t0, kc.cs, Ls);
                lagrange<T, PA>((double)t1, kc.ca, Lt);
                lagrange<T, PA>((double)t2, kc.ca, Lpp);
                cpx<T> val[RB];
                interp<T, PS, PA, RB>(&cone[pos * P * RB], Ls, Lt, Lpp, val);
                const T gr = g0, gim = conj_sign * g1;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    acc[r].x += val[r].x * gr - val[r].y * gim;
                    acc[r].y += val[r].x * gim + val[r].y * gr;
                }
            }
        }
        __syncthreads();
    }
    if (active) {
#pragma unroll
        for (int r = 0; r < RB; ++r) Fp[((size_t)sp * P + nu) * RB + r] = acc[r];
    }
}

// Capacity (cones) of the LDS stage: ~24 KB of cone values (48 KB for FP64
// with one right-hand side, whose cones are twice as large), at most
// S * kMaxFrameGroups.
template <typename T, int P, int RB, int S>
constexpr int lds_gcap()
{
    constexpr int bytes = (sizeof(T) == 8 && RB == 1) ? 49152 : 24576;
    return (bytes / (P * RB * (int)sizeof(cpx<T>))) < S * kMaxFrameGroups
               ? (bytes / (P * RB * (int)sizeof(cpx<T>)))
               : S * kMaxFrameGroups;
}

// Parent slots and threads per block of the LDS kernel: as many slots as fit
// 256 threads, at most 8.  (Blocks of 5 x 75 points in 384 threads, with
// 48 KB of staged cones, idle fewer lanes but ran 10% slower.)
template <int P, int RB>
constexpr int lds_slots()
{
    return (kBlock / P) < 8 ? (kBlock / P) : 8;
}

template <int P, int RB>
constexpr int lds_threads()
{
    return kBlock;
}

// Wavefronts per block of the per-slot matrix-core kernels: 4, fewer when the
// slots' accumulators (P x 2 RB values each) would pass 40 KB of LDS.
template <typename T, int P, int RB>
constexpr int mfma_waves()
{
    return (4 * P * 2 * RB * (int)sizeof(T) <= 40960) ? 4 : ((2 * P * 2 * RB * (int)sizeof(T) <= 40960) ? 2 : 1);
}

// Batched child-to-parent interpolation on the matrix cores (FP32, or FP64
// with the FP64 matrix instruction).  One wavefront handles one parent slot.
// For every child octant and every child cone ("group") the frame's
// interpolation points falling into that cone form the rows of 16 x 16 x 4
// MFMA tiles:
//   D[row][col] = sum_k A[row][k] B[k][col],
// A = the tensor Chebyshev weights of the row's point, B = the child cone's
// values, 2 RB real columns (re, im of RB right-hand sides) in tiles of 16.  The
// K index is ordered so that lane quarter q (lanes 16q..16q+15) always takes
// the phi-node c = q: its weights are Ls[a] Lt[b] Lp[q] with (a, b) fixed
// per step; the remaining phi-nodes c >= 4 follow in a short tail.  The
// re-centring ratio is applied per row and the result accumulated into the
// wavefront's own LDS copy of the slot's values, so no two wavefronts write
// the same data and the result does not depend on scheduling.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core product in the operand type: FP32
// (v_mfma_f32_16x16x4_f32) or FP64 (v_mfma_f64_16x16x4_f64).  Both take the
// operands as A[lane % 16][lane / 16] and B[lane / 16][lane % 16]; element i
// of the result holds D[row][lane % 16] with row = 4 (lane / 16) + i in FP32
// but row = lane / 16 + 4 i in FP64 (checked on the device: mfma_row).
template <typename T> struct MfmaVec;
template <> struct MfmaVec<float> { typedef mf4 type; };
template <> struct MfmaVec<double> { typedef md4 type; };
template <typename T>
using mvec = typename MfmaVec<T>::type;
__device__ inline mf4 mfma16(float a, float b, mf4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline md4 mfma16(double a, double b, md4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of element i of a 16 x 16 x 4 result in lane quarter q.
template <typename T>
__device__ inline int mfma_row(int q, int i)
{
    return sizeof(T) == 8 ? q + 4 * i : 4 * q + i;
}

// Tiles of CW columns: CW = 16 uses the 16 x 16 x 4 instruction; CW = 4 (FP64
// with at most 8 real columns) uses v_mfma_f64_4x4x4_4b_f64 with the four
// blocks as four groups of four rows sharing one B, which leaves no column
// of the instruction empty.  That instruction takes A[lane % 16][lane / 16]
// as the 16 x 16 x 4 one does and B[lane / 16][lane % 4], and returns row
// 4 ((lane % 16) / 4) + lane / 16, column lane % 4 (checked on the device);
// its FMA rate equals the 16 x 16 x 4 one's.
template <typename T, int CW>
using macc = typename std::conditional<CW == 16, mvec<T>, T>::type;

template <int CW, typename T>
__device__ inline macc<T, CW> mfma_step(T a, T b, macc<T, CW> c)
{
    if constexpr (CW == 16) {
        return mfma16(a, b, c);
    } else {
        static_assert(sizeof(T) == 8, "four-column tiles are FP64 only");
        return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
    }
}

// Row (within the tile) of output element i of this lane.
template <int CW, typename T>
__device__ inline int mfma_out_row(int lane, int i)
{
    if constexpr (CW == 16) return mfma_row<T>(lane >> 4, i);
    else return 4 * ((lane & 15) >> 2) + (lane >> 4);
}

// v[i] for a lane-dependent i, as a chain of selects on register values.
// The empty asm makes each element opaque, so the compiler cannot fold the
// chain back into an indexed load, which would move the array to scratch
// memory and make every use wait for all outstanding global loads.
template <int N, typename T>
__device__ inline T pick(const T* v, int i)
{
    T x = v[0];
#pragma unroll
    for (int j = 1; j < N; ++j) {
        T y = v[j];
        asm("" : "+v"(y));
        x = i == j ? y : x;
    }
    return x;
}

// One 16-row MFMA tile: rows are interpolation points of one child cone,
// columns the NC real values of the RB right-hand sides in NT tiles of 16.
// `b` holds the child cone's values as B operands (K ordering as described
// above); Ls/Lt/Lpv are the Chebyshev weights of this lane's row.
template <int PS, int PA, int NT, int CW = 16, typename T>
__device__ inline void mfma_tile(const T (*b)[PS * PA + (PS * PA * (PA - 4) + 3) / 4], const T* Ls,
                                 const T* Lt, const T* Lpv, int q, macc<T, CW>* c)
{
    constexpr int NAB = PS * PA;
    constexpr int NREM = NAB * (PA - 4);
    constexpr int KTAIL = (NREM + 3) / 4;
    const T lq = pick<4>(Lpv, q);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if constexpr (CW == 16) c[t] = mvec<T>{(T)0, (T)0, (T)0, (T)0};
        else c[t] = (T)0;
    }
    // the (s, theta) products, kept for the tail
    T pab[NAB];
#pragma unroll
    for (int ab = 0; ab < NAB; ++ab) {
        const int a = ab / PA, bb = ab - a * PA;
        pab[ab] = Ls[a] * Lt[bb];
        const T w = pab[ab] * lq;
#pragma unroll
        for (int t = 0; t < NT; ++t) c[t] = mfma_step<CW>(w, b[t][ab], c[t]);
    }
    // tail step jt: lane quarter q takes node (ab, c) = (m / (PA - 4),
    // 4 + m % (PA - 4)), m = 4 jt + q, so its product is one of at most four
    // consecutive entries of pab (from index lo) and one of the PA - 4 last
    // phi weights
#pragma unroll
    for (int jt = 0; jt < KTAIL; ++jt) {
        const int m = 4 * jt + q;
        constexpr int R = PA - 4;
        const int lo = (4 * jt) / R;
        const int abm = m / R, cc = m - abm * R;
        T w = (T)0;
        if (m < NREM) {
            const int span = (4 * jt + 3) / R - lo + 1;
            T pv = pab[lo];
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                if (j < span && lo + j < NAB) {
                    T y = pab[lo + j];
                    asm("" : "+v"(y));
                    pv = abm - lo == j ? y : pv;
                }
            }
            w = pv * pick<R>(Lpv + 4, cc);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) c[t] = mfma_step<CW>(w, b[t][NAB + jt], c[t]);
    }
}

// B operands of a child cone: lane (q, col) takes K entries (a, b, c = q)
// and the tail entries c >= 4, column 16 t + col of every tile t.
template <int PS, int PA, int NC, int NT, int CW = 16, typename T>
__device__ inline void mfma_load_b(const T* __restrict__ Fcs, int q, int col,
                                   T (*b)[PS * PA + (PS * PA * (PA - 4) + 3) / 4])
{
    constexpr int NAB = PS * PA;
    constexpr int NREM = NAB * (PA - 4);
    constexpr int KTAIL = (NREM + 3) / 4;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int cg = CW * t + col;
        const bool ok = cg < NC;
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) b[t][ab] = ok ? Fcs[(size_t)(ab * PA + q) * NC + cg] : (T)0;
#pragma unroll
        for (int jt = 0; jt < KTAIL; ++jt) {
            const int m = 4 * jt + q;
            T v = (T)0;
            if (ok && m < NREM) {
                const int abm = m / (PA - 4), cc = 4 + (m - abm * (PA - 4));
                v = Fcs[(size_t)(abm * PA + cc) * NC + cg];
            }
            b[t][NAB + jt] = v;
        }
    }
}

// Epilogue of a tile: rows mfma_row(q, i), column col of each tile; multiply by the
// row's ratio (complex: columns 2r, 2r+1 are re, im of right-hand side r) and
// accumulate into the wavefront's LDS values of the parent slot.
template <int NC, int NT, int CW = 16, typename T, typename I>
__device__ inline void mfma_epilogue(const macc<T, CW>* c, int lane, int t0, int cnt, const I* rownode,
                                     const T* ratio_re, const T* ratio_im, T* acc)
{
    const int col = lane % CW;
#pragma unroll
    for (int i = 0; i < (CW == 16 ? 4 : 1); ++i) {
        const int ri = t0 + mfma_out_row<CW, T>(lane, i);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            T v;
            if constexpr (CW == 16) v = c[t][i];
            else v = c[t];
            const T pv = __shfl_xor(v, 1, 64);
            const int cg = CW * t + col;
            if (ri < cnt && cg < NC) {
                const int nu = rownode[ri];
                const T gr = ratio_re[ri], gi = ratio_im[ri];
                const T o = (col & 1) == 0 ? v * gr - pv * gi : pv * gi + v * gr;
                acc[nu * NC + cg] += o;
            }
        }
    }
}

template <typename T, int PS, int PA, int RB, int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? (RB >= 16 ? 1 : 2) : (RB >= 16 ? 3 : 4))))
k_child_to_parent_mfma(KernelConsts kc, LevelDev Lc, LevelDev Lp, const cpx<T>* __restrict__ Fc,
                       cpx<T>* __restrict__ Fp)
{
    constexpr int P = PS * PA * PA;
    constexpr int NC = 2 * RB;                 // real columns
    constexpr int CW = 16;                     // columns per tile (the prefetched
                                               // operands of four-column tiles would spill)
    constexpr int NT = (NC + CW - 1) / CW;     // tiles
    constexpr int G = kMaxFrameGroups;
    constexpr int NK = PS * PA + (PS * PA * (PA - 4) + 3) / 4;
    static_assert(PA >= 4, "the K ordering needs at least four phi nodes");
    __shared__ T accs[W][P * NC];
    constexpr int ME = 64;                     // entries looked up at once
    __shared__ int sgo[W][9];                  // first entry of each octant
    __shared__ int entcs[W][ME];               // child slot of the entry, -1 missing
    __shared__ int entf[W][ME];                // its frame
    __shared__ int entr[W][ME];                // its rows: first | count << 8 (group order)
    __shared__ int rown[W][P];                 // point of each row of the current group
    __shared__ T rre[W][P], rim[W][P];         // its ratio
    __shared__ T rts[W][P], rtt[W][P], rtp[W][P];  // its local coordinates

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int sp = xcd_block(blockIdx.x, gridDim.x) * W + wv;
    if (sp >= Lp.nslots) return;               // whole wavefront leaves; no block barriers below
    T* acc = accs[wv];
    for (int i = lane; i < P * NC; i += 64) acc[i] = (T)0;

    const T* F = (const T*)Fc;
    const T* frt = (const T*)Lc.fr_t;
    const T* frr = (const T*)Lc.fr_ratio;
    const T conj_sign = kc.adj ? (T)-1 : (T)1;
    const int row = lane & 15, q = lane >> 4, col = lane % CW;
    const int j = Lp.slot_box[sp];

    // entries (octant, group) of this slot: lanes 0..7 hold the octants
    int fo = -1, ngo = 0;
    if (lane < 8) {
        fo = Lc.pframe[(size_t)sp * 8 + lane];
        ngo = fo >= 0 ? Lc.fr_ngrp[fo] : 0;
    }
    int incl = ngo;
#pragma unroll
    for (int dd = 1; dd < 8; dd <<= 1) {
        int y = __shfl_up(incl, dd, 64);
        if (lane >= dd) incl += y;
    }
    const int nent = __shfl(incl, 7, 64);
    if (lane < 8) sgo[wv][lane] = incl - ngo;
    if (lane == 0) sgo[wv][8] = nent;
    wave_lds_fence();

    // loads of entry e: B operands (raw) and its rows' point data; those of
    // the next entry are issued while the current entry's tiles run
    constexpr int RPL = (P + 63) / 64;
    T bn[NT][NK];
    int pn[RPL];
    T pt[RPL][3], pg[RPL][2];
    auto fetch = [&](int e) {
        const int f = entf[wv][e];
        const int cs = entcs[wv][e];
        mfma_load_b<PS, PA, NC, NT, CW>(F + (size_t)(cs >= 0 ? cs : 0) * P * NC, q, col, bn);
        const uint8_t* ord = Lc.fr_order + (size_t)f * P;
        const int g0 = entr[wv][e] & 255, cnt = entr[wv][e] >> 8;
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            int r = lane + 64 * h;
            r = r < cnt ? r : 0;
            const int nu = ord[g0 + r];
            const size_t ee = (size_t)f * P + nu;
            pn[h] = nu;
            pt[h][0] = frt[3 * ee];
            pt[h][1] = frt[3 * ee + 1];
            pt[h][2] = frt[3 * ee + 2];
            pg[h][0] = frr[2 * ee];
            pg[h][1] = frr[2 * ee + 1];
        }
    };
    for (int e0 = 0; e0 < nent; e0 += ME) {
    const int ne = nent - e0 < ME ? nent - e0 : ME;
    for (int e = lane; e < ne; e += 64) {
        const int E = e0 + e;
        int o = 0;
#pragma unroll
        for (int oo = 1; oo < 8; ++oo) o = sgo[wv][oo] <= E ? oo : o;
        const int g = E - sgo[wv][o];
        const int f = Lc.pframe[(size_t)sp * 8 + o];
        const int k = Lc.child_of[(size_t)j * 8 + o];
        const unsigned key = Lc.fr_gkey[(size_t)f * G + g];
        const int cell = (int)(key / (unsigned)Lc.ns), is = (int)(key - (unsigned)cell * Lc.ns);
        entcs[wv][e] = lookup(Lc, k, cell, is);
        entf[wv][e] = f;
        const int g0 = Lc.fr_goff[(size_t)f * (G + 1) + g], g1 = Lc.fr_goff[(size_t)f * (G + 1) + g + 1];
        entr[wv][e] = g0 | ((g1 - g0) << 8);
    }
    wave_lds_fence();
    fetch(0);
    for (int e = 0; e < ne; ++e) {
        const int cs = entcs[wv][e];
        const int cnt = entr[wv][e] >> 8;
        T b[NT][NK];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int k = 0; k < NK; ++k) b[t][k] = bn[t][k];
        // rows of the group: their points, local coordinates and ratios
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            const int r = lane + 64 * h;
            if (r < cnt) {
                rown[wv][r] = pn[h];
                rts[wv][r] = pt[h][0];
                rtt[wv][r] = pt[h][1];
                rtp[wv][r] = pt[h][2];
                rre[wv][r] = pg[h][0];
                rim[wv][r] = conj_sign * pg[h][1];
            }
        }
        if (e + 1 < ne) fetch(e + 1);
        if (cs < 0) {
            if (lane == 0) atomicAdd(kc.miss, (unsigned long long)cnt);
            wave_lds_fence();
            continue;
        }
        wave_lds_fence();
        for (int t0 = 0; t0 < cnt; t0 += 16) {
            T Ls[PS], Lt[PA], Lpv[PA];
            const int rr = t0 + row;
            const int rc = rr < cnt ? rr : 0;
            lagrange<T, PS>((double)rts[wv][rc], kc.cs, Ls);
            lagrange<T, PA>((double)rtt[wv][rc], kc.ca, Lt);
            lagrange<T, PA>((double)rtp[wv][rc], kc.ca, Lpv);
            if (rr >= cnt) {
#pragma unroll
                for (int i = 0; i < PS; ++i) Ls[i] = (T)0;
            }
            macc<T, CW> c[NT];
            mfma_tile<PS, PA, NT, CW>(b, Ls, Lt, Lpv, q, c);
            mfma_epilogue<NC, NT, CW>(c, lane, t0, cnt, rown[wv], rre[wv], rim[wv], acc);
        }
        wave_lds_fence();
    }
    }
    T* out = (T*)(Fp + (size_t)sp * P * RB);
    for (int i = lane; i < P * NC; i += 64) out[i] = acc[i];
}

// The same on levels without tabulated frames: every lane computes the
// child-frame geometry of interpolation points in FP64 (as k_child_to_parent
// does).  The (octant, point) pairs of the slot's children are taken in
// chunks of CH consecutive pairs, so the lanes stay busy when a frame's P
// points do not fill whole passes of 64; the wavefront sorts a chunk's
// points by (octant, child cone) with ballots ("groups"), looks the groups'
// cones up in parallel (one lane per group), and runs the groups' MFMA
// tiles.  Every point of an octant is in one group, and the groups come in
// octant order, so each parent point receives its octants' terms in octant
// order.  In FP32 up to 4 right-hand sides the kernel is held to 128 VGPRs,
// four wavefronts per SIMD instead of three: 15% faster.  (Loading the next
// group's operands during the current group's tiles was measured no faster
// in FP32 at 4 RHS, and in FP64 its registers cost a wave per SIMD; FP64 in
// 16 x 16 x 4 tiles, half of each unused, fits three wavefronts per SIMD
// but measured 5-6% slower.)
template <typename T, int PS, int PA, int RB, int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && RB <= 4 ? 4 : 1)))
k_child_to_parent_mfma_geo(KernelConsts kc, LevelDev Lc, LevelDev Lp,
                                                                      const cpx<T>* __restrict__ Fc,
                                                                      cpx<T>* __restrict__ Fp)
{
    constexpr int P = PS * PA * PA;
    constexpr int NC = 2 * RB;
    constexpr int CW = (sizeof(T) == 8 && NC <= 8) ? 4 : 16;   // columns per tile
    constexpr int NT = (NC + CW - 1) / CW;
    constexpr int NK = PS * PA + (PS * PA * (PA - 4) + 3) / 4;
    // lane passes per chunk (one with 16 right-hand sides, whose
    // accumulators leave less LDS)
    constexpr int NH = RB >= 16 ? 1 : 3;
    constexpr int CH = 64 * NH;                // (octant, point) pairs per chunk
    static_assert(PA >= 4, "the K ordering needs at least four phi nodes");
    static_assert(P <= 128, "point indices");
    __shared__ T accs[W][P * NC];
    __shared__ T rts[W][CH][3];                // local coordinates, in group order
    __shared__ T rre[W][CH], rim[W][CH];       // ratios, in group order
    __shared__ uint8_t rown[W][CH];            // parent point of each row
    __shared__ unsigned gkey[W][CH];           // child cone of each group
    __shared__ uint8_t goct[W][CH];            // octant of each group
    __shared__ int16_t goff[W][CH + 1];        // first row of each group
    __shared__ int gcs[W][CH];                 // child slot of each group, -1 missing

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int sp = xcd_block(blockIdx.x, gridDim.x) * W + wv;
    if (sp >= Lp.nslots) return;
    T* acc = accs[wv];
    for (int i = lane; i < P * NC; i += 64) acc[i] = (T)0;

    const T* F = (const T*)Fc;
    const int row = lane & 15, q = lane >> 4, col = lane % CW;
    const int j = Lp.slot_box[sp];
    const int pcone = Lp.slot_cone[sp];
    const int pcell = pcone / Lp.ns, pis = pcone - pcell * Lp.ns;
    const double half = 0.5 * Lc.H;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    // the octants with a child, in order, packed 4 bits each
    unsigned olist = 0;
    int m = 0;
    for (int o = 0; o < 8; ++o)
        if (Lc.child_of[(size_t)j * 8 + o] >= 0) olist |= (unsigned)o << (4 * m++);
    const int E = m * P;

    for (int c0 = 0; c0 < E; c0 += CH) {
        // geometry of the pairs c0 + lane + 64 h
        unsigned key[NH];
        int oi[NH];
        T tl[NH][3], gr[NH], gi[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int e = c0 + lane + 64 * h;
            key[h] = 0xffffffffu;
            oi[h] = -1;
            if (e < E) {
                const int ii = e / P, nu = e - ii * P;
                const int o = (int)((olist >> (4 * ii)) & 15u);
                oi[h] = ii;
                const double ov[3] = {(o & 1) ? half : -half, (o & 2) ? half : -half, (o & 4) ? half : -half};
                const int a = nu / (PA * PA), bc = nu - a * PA * PA;
                const double rr = Lp.node_r[pis * PS + a];
                const double* dir = &Lp.node_dir[((size_t)pcell * PA * PA + bc) * 3];
                const double y0 = rr * dir[0], y1 = rr * dir[1], y2 = rr * dir[2];
                const double ry = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
                double v[3];
                node_minus(rr, dir, ov, v);
                ConeLoc cl;
                cone_locate(v[0], v[1], v[2], Lc.h, Lc.ds, Lc.dang, Lc.ns, Lc.nc, cl);
                key[h] = (unsigned)(cl.cell * Lc.ns + cl.is);
                tl[h][0] = (T)cl.ts;
                tl[h][1] = (T)cl.tt;
                tl[h][2] = (T)cl.tp;
                const double num = (ov[0] * ov[0] + ov[1] * ov[1] + ov[2] * ov[2]) -
                                   2.0 * (y0 * ov[0] + y1 * ov[1] + y2 * ov[2]);
                const double diff = num / (cl.r + ry);
                T cph, sph;
                expi<T>(kc.kappa * diff, cph, sph);
                const T mag = (T)(ry / cl.r);
                gr[h] = mag * cph;
                gi[h] = mag * sph;
            } else {
                tl[h][0] = tl[h][1] = tl[h][2] = gr[h] = gi[h] = (T)0;
            }
        }
        // the groups: pairs sorted by (octant, child cone), in order of first
        // appearance
        bool un[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) un[h] = oi[h] >= 0;
        int ng = 0, base = 0;
        for (;;) {
            unsigned long long mk[NH];
            int leader = -1;
#pragma unroll
            for (int h = NH - 1; h >= 0; --h) {
                mk[h] = __ballot(un[h]);
                if (mk[h]) leader = 64 * h + (__ffsll((long long)mk[h]) - 1);
            }
            if (leader < 0) break;
            unsigned lk = 0;
            int lo = 0;
#pragma unroll
            for (int h = 0; h < NH; ++h)
                if (leader / 64 == h) {
                    lk = __shfl(key[h], leader & 63, 64);
                    lo = __shfl(oi[h], leader & 63, 64);
                }
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const bool in = un[h] && key[h] == lk && oi[h] == lo;
                const unsigned long long g = __ballot(in);
                if (in) {
                    const int r = base + __popcll(g & lt_mask);
                    const int e = c0 + lane + 64 * h;
                    rown[wv][r] = (uint8_t)(e - oi[h] * P);
                    rts[wv][r][0] = tl[h][0];
                    rts[wv][r][1] = tl[h][1];
                    rts[wv][r][2] = tl[h][2];
                    rre[wv][r] = gr[h];
                    rim[wv][r] = gi[h];
                }
                un[h] = un[h] && !in;
                if (lane == 0 && h == 0) {
                    gkey[wv][ng] = lk;
                    goct[wv][ng] = (uint8_t)((olist >> (4 * lo)) & 15u);
                    goff[wv][ng] = (int16_t)base;
                }
                base += __popcll(g);
            }
            ++ng;
        }
        if (lane == 0) goff[wv][ng] = (int16_t)base;
        wave_lds_fence();
        // the groups' child slots, looked up together
        for (int g = lane; g < ng; g += 64) {
            const unsigned kk = gkey[wv][g];
            const int cell = (int)(kk / (unsigned)Lc.ns), is = (int)(kk - (unsigned)cell * Lc.ns);
            const int cs = lookup(Lc, Lc.child_of[(size_t)j * 8 + goct[wv][g]], cell, is);
            gcs[wv][g] = cs;
            if (cs < 0) atomicAdd(kc.miss, (unsigned long long)(goff[wv][g + 1] - goff[wv][g]));
        }
        wave_lds_fence();
        // the tiles, group by group
        for (int g = 0; g < ng; ++g) {
            const int cs = gcs[wv][g];
            if (cs < 0) continue;
            T b[NT][NK];
            mfma_load_b<PS, PA, NC, NT, CW>(F + (size_t)cs * P * NC, q, col, b);
            const int g0 = goff[wv][g], cnt = goff[wv][g + 1] - g0;
            for (int t0 = 0; t0 < cnt; t0 += 16) {
                T Ls[PS], Lt[PA], Lpv[PA];
                const int rr = t0 + row;
                if (rr < cnt) {
                    const T* tr = rts[wv][g0 + rr];
                    lagrange<T, PS>((double)tr[0], kc.cs, Ls);
                    lagrange<T, PA>((double)tr[1], kc.ca, Lt);
                    lagrange<T, PA>((double)tr[2], kc.ca, Lpv);
                } else {
#pragma unroll
                    for (int i = 0; i < PS; ++i) Ls[i] = (T)0;
#pragma unroll
                    for (int i = 0; i < PA; ++i) Lt[i] = Lpv[i] = (T)0;
                }
                macc<T, CW> c[NT];
                mfma_tile<PS, PA, NT, CW>(b, Ls, Lt, Lpv, q, c);
                mfma_epilogue<NC, NT, CW>(c, lane, t0, cnt, &rown[wv][g0], &rre[wv][g0], &rim[wv][g0], acc);
            }
        }
        wave_lds_fence();
    }
    T* out = (T*)(Fp + (size_t)sp * P * RB);
    for (int i = lane; i < P * NC; i += 64) out[i] = acc[i];
}

constexpr int kQuadSlots = 12;    // parent slots per block of the quad kernel

// Child cones staged at once by the quad kernel: about 24 KB.
template <typename T, int P>
constexpr int quad_gcap()
{
    return 24576 / (P * (int)sizeof(cpx<T>)) < 4 ? 4 : 24576 / (P * (int)sizeof(cpx<T>));
}

// Child-to-parent interpolation, one right-hand side, on the vector units,
// with each child cone value read from LDS once for up to QR interpolation
// points.  A block handles S consecutive parent slots, octant by octant: the
// child cones of the octant's (slot, group) entries are staged in LDS, and
// every thread takes a "quad" -- up to QR consecutive points of one group in
// the frame's group order -- and contracts the cone one direction at a time
// (phi, then theta, then s) for all its points together.  The points' values,
// times the re-centring ratio, are added to the slot's accumulators in LDS
// (each (slot, point) belongs to one quad per octant, so no two threads touch
// the same accumulator in a step).
template <typename T, int PS, int PA, int S, int QR, int GCAP>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
k_child_to_parent_quads(KernelConsts kc, LevelDev Lc, LevelDev Lp,
                                                                  const cpx<T>* __restrict__ Fc,
                                                                  cpx<T>* __restrict__ Fp)
{
    constexpr int P = PS * PA * PA;
    constexpr int G = kMaxFrameGroups;
    constexpr int MAXE = S * G;
    static_assert(S <= 64, "slots of a block are scanned in one wavefront");
    __shared__ cpx<T> cone[GCAP * P];
    __shared__ cpx<T> acc[S * P];
    __shared__ int sfr[S];             // frame of (slot, octant), -1
    __shared__ int soff[S + 1];        // first entry of each slot
    __shared__ int qoff[S + 1];        // first quad of each slot
    __shared__ int staged[MAXE];       // child slot of each entry, -1 missing

    const int tid = threadIdx.x;
    const int slot0 = xcd_block(blockIdx.x, gridDim.x) * S;
    const T* frt = (const T*)Lc.fr_t;
    const T* frr = (const T*)Lc.fr_ratio;
    const T conj_sign = kc.adj ? (T)-1 : (T)1;
    for (int i = tid; i < S * P; i += kBlock) acc[i] = cpx<T>{(T)0, (T)0};

    for (int o = 0; o < 8; ++o) {
        // frames, entry and quad counts of the slots, exclusive scans
        if (tid < 64) {
            int f = -1, ng = 0, nq = 0;
            if (tid < S && slot0 + tid < Lp.nslots) {
                f = Lc.pframe[(size_t)(slot0 + tid) * 8 + o];
                if (f >= 0) {
                    ng = Lc.fr_ngrp[f];
                    const uint8_t* go = Lc.fr_goff + (size_t)f * (G + 1);
                    for (int g = 0; g < ng; ++g) nq += (go[g + 1] - go[g] + QR - 1) / QR;
                }
            }
            int xe = ng, xq = nq;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const int ye = __shfl_up(xe, dd, 64), yq = __shfl_up(xq, dd, 64);
                if (tid >= dd) {
                    xe += ye;
                    xq += yq;
                }
            }
            if (tid < S) {
                sfr[tid] = f;
                soff[tid + 1] = xe;
                qoff[tid + 1] = xq;
            }
            if (tid == 0) soff[0] = qoff[0] = 0;
        }
        __syncthreads();
        const int nent = soff[S], nquad = qoff[S];
        for (int i = tid; i < nent; i += kBlock) {
            int sl = 0;
            while (soff[sl + 1] <= i) ++sl;
            const int g = i - soff[sl], f = sfr[sl];
            const int k = Lc.child_of[(size_t)Lp.slot_box[slot0 + sl] * 8 + o];
            const unsigned key = Lc.fr_gkey[(size_t)f * G + g];
            const int cell = (int)(key / (unsigned)Lc.ns), is = (int)(key - (unsigned)cell * Lc.ns);
            const int cs = k >= 0 ? lookup(Lc, k, cell, is) : -1;
            staged[i] = cs;
        }
        __syncthreads();
        for (int base = 0; base < nent; base += GCAP) {
            const int cnt = nent - base < GCAP ? nent - base : GCAP;
            for (int i = tid; i < cnt * P; i += kBlock) {
                const int q = i / P, off = i - q * P;
                const int cs = staged[base + q];
                if (cs >= 0) cone[i] = Fc[(size_t)cs * P + off];
            }
            __syncthreads();
            for (int qi = tid; qi < nquad; qi += kBlock) {
                int sl = 0;
                while (qoff[sl + 1] <= qi) ++sl;
                const int f = sfr[sl];
                const uint8_t* go = Lc.fr_goff + (size_t)f * (G + 1);
                int rest = qi - qoff[sl], g = 0;
                for (;;) {
                    const int nqg = (go[g + 1] - go[g] + QR - 1) / QR;
                    if (rest < nqg) break;
                    rest -= nqg;
                    ++g;
                }
                const int ent = soff[sl] + g;
                if (ent < base || ent >= base + cnt) continue;
                const int r0 = go[g] + rest * QR;
                const int nr = go[g + 1] - r0 < QR ? go[g + 1] - r0 : QR;
                if (staged[ent] < 0) {
                    atomicAdd(kc.miss, (unsigned long long)nr);
                    continue;
                }
                const uint8_t* ord = Lc.fr_order + (size_t)f * P;
                int nu[QR];
                T Ls[QR][PS], Lt[QR][PA], Lq[QR][PA];
#pragma unroll
                for (int r = 0; r < QR; ++r) {
                    nu[r] = ord[r0 + (r < nr ? r : 0)];
                    const size_t e = (size_t)f * P + nu[r];
                    lagrange<T, PS>((double)frt[3 * e], kc.cs, Ls[r]);
                    lagrange<T, PA>((double)frt[3 * e + 1], kc.ca, Lt[r]);
                    lagrange<T, PA>((double)frt[3 * e + 2], kc.ca, Lq[r]);
                }
                const cpx<T>* F = &cone[(ent - base) * P];
                cpx<T> U[QR][PS];
#pragma unroll
                for (int r = 0; r < QR; ++r)
#pragma unroll
                    for (int a = 0; a < PS; ++a) U[r][a] = cpx<T>{(T)0, (T)0};
                // one phi-row of the cone per step, the next one loaded ahead;
                // the empty asm keeps the compiler from hoisting all loads
                cpx<T> fv[PA], fn[PA];
#pragma unroll
                for (int c = 0; c < PA; ++c) fv[c] = F[c];
#pragma unroll
                for (int ab = 0; ab < PS * PA; ++ab) {
                    const int a = ab / PA, b = ab - a * PA;
                    if (ab + 1 < PS * PA) {
#pragma unroll
                        for (int c = 0; c < PA; ++c) fn[c] = F[(ab + 1) * PA + c];
                    }
                    asm volatile("" ::: "memory");
#pragma unroll
                    for (int r = 0; r < QR; ++r) {
                        T sr = (T)0, si = (T)0;
#pragma unroll
                        for (int c = 0; c < PA; ++c) {
                            sr += fv[c].x * Lq[r][c];
                            si += fv[c].y * Lq[r][c];
                        }
                        U[r][a].x += sr * Lt[r][b];
                        U[r][a].y += si * Lt[r][b];
                    }
#pragma unroll
                    for (int c = 0; c < PA; ++c) fv[c] = fn[c];
                }
#pragma unroll
                for (int r = 0; r < QR; ++r) {
                    if (r < nr) {
                        T vr = (T)0, vi = (T)0;
#pragma unroll
                        for (int a = 0; a < PS; ++a) {
                            vr += U[r][a].x * Ls[r][a];
                            vi += U[r][a].y * Ls[r][a];
                        }
                        const size_t e = (size_t)f * P + nu[r];
                        const T gr = frr[2 * e], gi = conj_sign * frr[2 * e + 1];
                        cpx<T>& A = acc[sl * P + nu[r]];
                        A.x += vr * gr - vi * gi;
                        A.y += vr * gi + vi * gr;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < S * P; i += kBlock) {
        const int sl = i / P;
        if (slot0 + sl < Lp.nslots) Fp[(size_t)slot0 * P + i] = acc[i];
    }
}


// Child-to-parent interpolation batched over boxes on the matrix cores
// (FP32).  A frame depends only on the parent cone and the octant, so the
// interpolation weights of a (frame, child cone) group are the same in every
// box that holds the parent cone.  A box tile lists up to kBoxTile parent
// slots of one parent cone; one wavefront runs, for every (octant, group)
// entry, 16 x 16 x 4 MFMA tiles whose rows are the group's interpolation
// points, K the child cone's nodes (ordered as in mfma_tile) and columns
// (box, right-hand side, re / im), two 16-column tiles per pass: BX boxes per
// pass, the tile's slots in ceil(n / BX) passes.
//   Per octant, the frame's points are staged once (the products
// Ls[a] Lt[b] and Lp[c] of every point, its re-centring ratio), the tiles
// store their raw results in LDS, and one combine step multiplies them by the
// ratio into accumulators held in registers: lane (ph, cc) owns complex
// column cc and the points nu = ph + 4k.  The tile's entries and the child
// slot each reads in each box come from tables the plan built, so a chunk of
// entries is read in one step; the B operands of the next entry and the
// points of the next octant are loaded while the current tiles run.  Each
// parent slot is written by exactly one wavefront.
constexpr int kBoxMaxEnt = 40;    // (octant, group) entries read at once
constexpr int kCompactEnt = 24;   // the same for the compact FP64 box kernel, whose frames
                                  // may touch at most this many child cones

template <int PS, int PA, int RB>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_child_to_parent_boxes(KernelConsts kc, LevelDev Lc, LevelDev Lp, const cpx<float>* __restrict__ Fc,
                        cpx<float>* __restrict__ Fp, const cpx<float>* __restrict__ zero_cone)
{
    constexpr int P = PS * PA * PA;
    constexpr int NT = 2;                      // tiles per pass: real and imaginary parts
    static_assert(16 % RB == 0, "a pass holds whole boxes");
    constexpr int BX = 16 / RB;                // boxes per pass (16 complex columns)
    constexpr int AS = 33;                     // row stride of the raw results (odd: LDS banks)
    constexpr int G = kMaxFrameGroups;
    constexpr int ME = kBoxMaxEnt;
    constexpr int NAB = PS * PA;
    constexpr int NREM = NAB * (PA - 4);
    constexpr int NK = NAB + (NREM + 3) / 4;
    constexpr int WS = NAB + PA + 1;           // staged weights per point (odd stride: LDS banks)
    constexpr int RPL = (P + 63) / 64;         // points per lane when staging
    constexpr int KC = (P + 3) / 4;            // points per lane in the combine
    static_assert(PA >= 4, "the K ordering needs at least four phi nodes");
    static_assert(P <= 255 && ME >= G, "entry and point indices");
    __shared__ float tmp[P * AS];              // raw tile results (re | im) by group position
    __shared__ float wts[P * WS];              // Ls[a] Lt[b] (ab < NAB), then Lp[c], by group position
    __shared__ float srat[P][2];               // ratio of point nu
    __shared__ uint8_t spos[P];                // group position of point nu
    __shared__ uint8_t sord[8 * P];            // points of the 8 frames in group order
    __shared__ int sfr[8];                     // frame of each octant, -1
    __shared__ int sgo[9];                     // first entry of each octant
    __shared__ int bslot[kBoxTile];
    __shared__ uint8_t smask[kBoxTile];        // children of each tile box (bit o)
    __shared__ int einfo[ME];                  // g0 | cnt << 8 | o << 16
    __shared__ int ecs[ME * BX];               // child slot of (entry, box of the pass), -1

    const int lane = threadIdx.x;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    if (tile >= Lc.ntiles) return;
    const float* frt = (const float*)Lc.fr_t;
    const float* frr = (const float*)Lc.fr_ratio;
    const float conj_sign = kc.adj ? -1.f : 1.f;
    const int row = lane & 15, q = lane >> 4, col = lane & 15;
    const int cc = lane & 15, ph = lane >> 4;  // combine: complex column, point phase

    // the tile's slots, their boxes' children, the octants' frames and the
    // tile's entries (tabulated by the plan)
    int my_slot = -1;
    if (lane < kBoxTile) {
        my_slot = Lc.bt_slot[(size_t)tile * kBoxTile + lane];
        bslot[lane] = my_slot;
        smask[lane] = Lc.te_mask[(size_t)tile * kBoxTile + lane];
    }
    if (lane < 8) sfr[lane] = Lc.bt_frame[(size_t)tile * 8 + lane];
    if (lane < 9) sgo[lane] = Lc.te_go[(size_t)tile * 9 + lane];
    const int64_t ebase = Lc.te_start[tile];
    const int nbt = __popcll(__ballot(my_slot >= 0));
    wave_lds_fence();
    for (int i = lane; i < 8 * P; i += 64) {
        const int o = i / P, r = i - o * P;
        const int f = sfr[o];
        const uint8_t v = Lc.fr_order[(size_t)(f >= 0 ? f : 0) * P + r];
        sord[i] = f >= 0 ? v : (uint8_t)0;
    }
    wave_lds_fence();

    // point data of an octant's frame (by group position r = lane + 64 h)
    int pn[RPL];
    float pt[RPL][3], pg[RPL][2];
    auto fetch_points = [&](int o) {
        const int f = sfr[o];
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            int r = lane + 64 * h;
            r = r < P ? r : 0;
            const int nu = sord[o * P + r];
            const size_t ee = (size_t)(f >= 0 ? f : 0) * P + nu;
            pn[h] = nu;
            pt[h][0] = frt[3 * ee];
            pt[h][1] = frt[3 * ee + 1];
            pt[h][2] = frt[3 * ee + 2];
            pg[h][0] = frr[2 * ee];
            pg[h][1] = frr[2 * ee + 1];
        }
    };
    // B operands of an entry: column col is (box col / RB, right-hand side
    // col % RB); tile 0 takes the real parts, tile 1 the imaginary parts, so
    // each value is one 8-byte load.  A missing child reads the zero cone.
    float bn[NT][NK];
    auto fetch_b = [&](int ei) {
        const int cs = ecs[ei * BX + col / RB];
        const cpx<float>* src = cs >= 0 ? Fc + (size_t)cs * P * RB + (col % RB) : zero_cone;
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) {
            const cpx<float> v = src[(size_t)(ab * PA + q) * RB];
            bn[0][ab] = v.x;
            bn[1][ab] = v.y;
        }
#pragma unroll
        for (int jt = 0; jt < NK - NAB; ++jt) {
            int m = 4 * jt + q;
            m = m < NREM ? m : NREM - 1;
            const int abm = m / (PA - 4), c4 = 4 + (m - abm * (PA - 4));
            const cpx<float> v = src[(size_t)(abm * PA + c4) * RB];
            bn[0][NAB + jt] = v.x;
            bn[1][NAB + jt] = v.y;
        }
    };

    for (int b0 = 0; b0 < nbt; b0 += BX) {
        float accr[KC], acci[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) accr[k] = acci[k] = 0.f;
        // octants in which a box of the pass has a child: the others would
        // only add products with the zero cone
        int pm = 0;
        if constexpr (BX == 16) {
            pm = 255;
        } else {
            const int bl = lane >> 3, o = lane & 7;
            const bool has = lane < BX * 8 && b0 + bl < kBoxTile && ((smask[b0 + bl] >> o) & 1);
            const unsigned long long bal = __ballot(has);
#pragma unroll
            for (int k = 0; k < BX; ++k) pm |= (int)((bal >> (8 * k)) & 255ull);
        }
        auto live = [&](int o) { return sfr[o] >= 0 && ((pm >> o) & 1); };
        int o0 = 0;
        while (o0 < 8) {
            // a chunk of whole octants with at most ME entries
            int o1 = o0 + 1;
            while (o1 < 8 && sgo[o1 + 1] - sgo[o0] <= ME) ++o1;
            const int e0 = sgo[o0], ne = sgo[o1] - e0;
            const int64_t eb = ebase + e0;
            for (int i = lane; i < ne; i += 64) einfo[i] = Lc.te_info[eb + i];
            for (int i = lane; i < ne * BX; i += 64) {
                const int ei = i / BX, bl = i - ei * BX;
                const int bi = b0 + bl;
                int cs = bi < kBoxTile ? Lc.te_cs[(size_t)(eb + ei) * kBoxTile + bi] : -1;
                if (cs == -2) {
                    atomicAdd(kc.miss, (unsigned long long)((Lc.te_info[eb + ei] >> 8) & 255));
                    cs = -1;
                }
                ecs[i] = cs;
            }
            wave_lds_fence();
            int o_pts = o0;
            while (o_pts < o1 && !live(o_pts)) ++o_pts;
            if (o_pts < o1) {
                // (with all boxes in the pass, octants without entries are
                // the only ones skipped, so the first live entry is 0)
                fetch_b(BX == 16 ? 0 : sgo[o_pts] - e0);
                fetch_points(o_pts);
            }
            int ei = 0;
            for (int o = o0; o < o1; ++o) {
                if (!live(o)) {
                    if constexpr (BX < 16) ei = sgo[o + 1] - e0;
                    continue;
                }
                // stage the frame's points: weights by group position, ratio and position by point
#pragma unroll
                for (int h = 0; h < RPL; ++h) {
                    const int r = lane + 64 * h;
                    if (r < P) {
                        float Ls[PS], Lt[PA], Lpv[PA];
                        lagrange<float, PS>((double)pt[h][0], kc.cs, Ls);
                        lagrange<float, PA>((double)pt[h][1], kc.ca, Lt);
                        lagrange<float, PA>((double)pt[h][2], kc.ca, Lpv);
                        float* w = &wts[r * WS];
#pragma unroll
                        for (int a = 0; a < PS; ++a)
#pragma unroll
                            for (int bb = 0; bb < PA; ++bb) w[a * PA + bb] = Ls[a] * Lt[bb];
#pragma unroll
                        for (int c4 = 0; c4 < PA; ++c4) w[NAB + c4] = Lpv[c4];
                        srat[pn[h]][0] = pg[h][0];
                        srat[pn[h]][1] = conj_sign * pg[h][1];
                        spos[pn[h]] = (uint8_t)r;
                    }
                }
                int on = o + 1;
                while (on < o1 && !live(on)) ++on;
                if (on < o1) fetch_points(on);
                wave_lds_fence();
                const int e_end = sgo[o + 1] - e0;
                // the entry after the octant's last: the next live octant's first
                const int e_next = on < o1 ? sgo[on] - e0 : ne;
                for (; ei < e_end; ++ei) {
                    const int info = einfo[ei];
                    const int g0 = info & 255, cnt = (info >> 8) & 255;
                    // the entry's operands, taken over from the prefetch (the
                    // empty asm makes them values of their own, so the wait
                    // for their loads falls here and not before every tile),
                    // then the loads of the next live entry (this entry's
                    // again after the last: a load on every path keeps the
                    // registers of both in place)
                    float b[NT][NK];
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int k = 0; k < NK; ++k) {
                            b[t][k] = bn[t][k];
                            asm volatile("" : "+v"(b[t][k]));
                        }
                    const int en = (BX == 16 || ei + 1 < e_end) ? ei + 1 : e_next;
                    fetch_b(en < ne ? en : ei);
                    for (int t0 = 0; t0 < cnt; t0 += 16) {
                        const int rr = t0 + row;
                        const int r = g0 + (rr < cnt ? rr : 0);
                        const float* w = &wts[r * WS];
                        const float z = rr < cnt ? 1.f : 0.f;
                        const float lq = w[NAB + q] * z;
                        mf4 c[NT];
#pragma unroll
                        for (int t = 0; t < NT; ++t) c[t] = mf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int ab = 0; ab < NAB; ++ab) {
                            const float wk = w[ab] * lq;
#pragma unroll
                            for (int t = 0; t < NT; ++t)
                                c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wk, b[t][ab], c[t], 0, 0, 0);
                        }
#pragma unroll
                        for (int jt = 0; jt < NK - NAB; ++jt) {
                            const int m = 4 * jt + q;
                            const int mm = m < NREM ? m : 0;
                            const int abm = mm / (PA - 4), c4 = 4 + (mm - abm * (PA - 4));
                            const float wk = m < NREM ? w[abm] * w[NAB + c4] * z : 0.f;
#pragma unroll
                            for (int t = 0; t < NT; ++t)
                                c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wk, b[t][NAB + jt], c[t], 0, 0, 0);
                        }
                        // rows 4q + i of the tile go to group positions g0 + t0 + 4q + i
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int ri = t0 + 4 * q + i;
                            if (ri < cnt) {
#pragma unroll
                                for (int t = 0; t < NT; ++t) tmp[(g0 + ri) * AS + 16 * t + col] = c[t][i];
                            }
                        }
                    }
                }
                wave_lds_fence();
                // combine: value times ratio into the register accumulators
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const int nu = ph + 4 * k;
                    if (nu < P) {
                        const int r = spos[nu];
                        const float vr = tmp[r * AS + cc], vi = tmp[r * AS + 16 + cc];
                        const float gr = srat[nu][0], gi = srat[nu][1];
                        accr[k] += vr * gr - vi * gi;
                        acci[k] += vr * gi + vi * gr;
                    }
                }
                wave_lds_fence();
            }
            o0 = o1;
        }
        // write the pass's slots: column cc is (box bl, right-hand side rr)
        const int bl = cc / RB, rr = cc - bl * RB;
        const int bi = b0 + bl;
        const int s = bi < kBoxTile ? bslot[bi] : -1;
        if (s >= 0) {
            cpx<float>* out = Fp + (size_t)s * P * RB + rr;
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const int nu = ph + 4 * k;
                if (nu < P) out[(size_t)nu * RB] = cpx<float>{accr[k], acci[k]};
            }
        }
    }
}

// Box-batched child-to-parent with the parent values accumulated in LDS
// (FP32 or FP64 matrix instructions).  Same tiles, entries and matrix
// shapes as k_child_to_parent_boxes -- one wavefront per tile of boxes that
// share a parent cone, 16 (box, right-hand side) columns per pass, rows =
// the points of one child cone ("group") of the octant's frame, K = the
// child cone's nodes -- but the wavefront keeps only the octant's local
// coordinates and ratios in LDS and forms each row's Chebyshev weights in
// registers, and the epilogue multiplies every raw result by its point's
// ratio and adds it to the pass's values in LDS (each (point, column)
// belongs to one lane of one tile in an octant, so there are no races).
// Without the raw-result and weight staging, FP64 fits in registers at two
// waves per SIMD (its LDS allows six waves per CU), FP32 at three.  The next
// live octant's frame is loaded while the current one runs, and an entry's
// B operands are loaded when the entry starts (a second operand set, loaded
// one entry ahead, measured slower for both types).
template <typename T, int PS, int PA, int RB, bool HALF, bool CMP = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HALF && sizeof(T) == 4 ? 4 : 3)))
k_child_to_parent_boxacc(KernelConsts kc, LevelDev Lc, LevelDev Lp, const cpx<T>* __restrict__ Fc,
                         cpx<T>* __restrict__ Fp, const cpx<T>* __restrict__ zero_cone)
{
    constexpr int P = PS * PA * PA;
    // HALF: a pass holds 8 complex columns as the 16 columns of one tile (real
    // and imaginary parts of a column side by side), so that the accumulators
    // take half the LDS; else 16 complex columns in two tiles, real parts in
    // tile 0 and imaginary parts in tile 1
    constexpr int CP = HALF ? 8 : 16;          // complex columns per pass
    constexpr int NT = HALF ? 1 : 2;           // tiles per pass
    static_assert(CP % RB == 0, "a pass holds whole boxes");
    constexpr int BX = CP / RB;                // boxes per pass
    // CMP (FP64, full width, levels whose frames touch at most kCompactEnt
    // child cones): the accumulators unpadded with their columns XOR-swizzled
    // by the point against bank conflicts, only the current octant's point
    // order in LDS (loaded one octant ahead with its frame), chunks of at most
    // kCompactEnt entries and the tile's slots and child masks in registers,
    // so that seven wavefronts fit per CU instead of six
    static_assert(!CMP || (!HALF && sizeof(T) == 8), "the compact layout is FP64 full width");
    constexpr int AS = CMP ? 32 : (HALF ? 17 : 33);   // row stride of the accumulators
    constexpr int ME = CMP ? kCompactEnt : kBoxMaxEnt;
    constexpr int NAB = PS * PA;
    constexpr int NREM = NAB * (PA - 4);
    constexpr int NK = NAB + (NREM + 3) / 4;
    static_assert(PA >= 4, "the K ordering needs at least four phi nodes");
    static_assert(P <= 255 && (CMP || ME >= kMaxFrameGroups), "entry and point indices");
    __shared__ T acc[P * AS];                  // the pass's parent values by point
    __shared__ T rt[3][P];                     // local coordinates of the octant's points
    __shared__ T rg[2][P];                     // their ratios
    __shared__ uint8_t sord[CMP ? P : 8 * P];  // points of the frames in group order (CMP: the octant's)
    __shared__ int sfr[8];                     // frame of each octant, -1
    __shared__ int sgo[9];                     // first entry of each octant
    __shared__ int bslot[CMP ? 1 : kBoxTile];
    __shared__ uint8_t smask[CMP ? 1 : kBoxTile];   // children of each tile box (bit o)
    __shared__ int einfo[ME];                  // g0 | cnt << 8 | o << 16
    __shared__ int ecs[ME * BX];               // child slot of (entry, box of the pass), -1

    const int lane = threadIdx.x;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    if (tile >= Lc.ntiles) return;
    const T* frt = (const T*)Lc.fr_t;
    const T* frr = (const T*)Lc.fr_ratio;
    const T conj_sign = kc.adj ? (T)-1 : (T)1;
    const int row = lane & 15, q = lane >> 4, col = lane & 15;

    int my_slot = -1, my_mask = 0;
    if (lane < kBoxTile) {
        my_slot = Lc.bt_slot[(size_t)tile * kBoxTile + lane];
        my_mask = Lc.te_mask[(size_t)tile * kBoxTile + lane];
        if constexpr (!CMP) {
            bslot[lane] = my_slot;
            smask[lane] = (uint8_t)my_mask;
        }
    }
    // accumulator of (point nu, column cc)
    auto aix = [&](int nu, int cc) { return CMP ? nu * AS + ((cc & 16) | ((cc ^ nu) & 15)) : nu * AS + cc; };
    if (lane < 8) sfr[lane] = Lc.bt_frame[(size_t)tile * 8 + lane];
    if (lane < 9) sgo[lane] = Lc.te_go[(size_t)tile * 9 + lane];
    const int64_t ebase = Lc.te_start[tile];
    const int nbt = __popcll(__ballot(my_slot >= 0));
    wave_lds_fence();
    if constexpr (!CMP) {
        for (int i = lane; i < 8 * P; i += 64) {
            const int o = i / P, r = i - o * P;
            const int f = sfr[o];
            const uint8_t v = Lc.fr_order[(size_t)(f >= 0 ? f : 0) * P + r];
            sord[i] = f >= 0 ? v : (uint8_t)0;
        }
    }
    wave_lds_fence();

    // B operands of an entry: column col is (box col / RB, right-hand side
    // col % RB); tile 0 takes the real parts, tile 1 the imaginary parts.  A
    // missing child reads the zero cone.
    T bn[NT][NK];
    auto fetch_b = [&](int ei) {
        if constexpr (HALF) {
            // column col: part col % 2 of complex column col / 2
            const int cc = col >> 1, part = col & 1;
            const int cs = ecs[ei * BX + cc / RB];
            const T* src = (const T*)(cs >= 0 ? Fc + (size_t)cs * P * RB + (cc % RB) : zero_cone + (cc % RB)) + part;
#pragma unroll
            for (int ab = 0; ab < NAB; ++ab) bn[0][ab] = src[(size_t)(ab * PA + q) * RB * 2];
#pragma unroll
            for (int jt = 0; jt < NK - NAB; ++jt) {
                int m = 4 * jt + q;
                m = m < NREM ? m : NREM - 1;
                const int abm = m / (PA - 4), c4 = 4 + (m - abm * (PA - 4));
                bn[0][NAB + jt] = src[(size_t)(abm * PA + c4) * RB * 2];
            }
        } else {
            const int cs = ecs[ei * BX + col / RB];
            const cpx<T>* src = cs >= 0 ? Fc + (size_t)cs * P * RB + (col % RB) : zero_cone + (col % RB);
#pragma unroll
            for (int ab = 0; ab < NAB; ++ab) {
                const cpx<T> v = src[(size_t)(ab * PA + q) * RB];
                bn[0][ab] = v.x;
                bn[NT - 1][ab] = v.y;
            }
#pragma unroll
            for (int jt = 0; jt < NK - NAB; ++jt) {
                int m = 4 * jt + q;
                m = m < NREM ? m : NREM - 1;
                const int abm = m / (PA - 4), c4 = 4 + (m - abm * (PA - 4));
                const cpx<T> v = src[(size_t)(abm * PA + c4) * RB];
                bn[0][NAB + jt] = v.x;
                bn[NT - 1][NAB + jt] = v.y;
            }
        }
    };

    for (int b0 = 0; b0 < nbt; b0 += BX) {
        for (int i = lane; i < P * AS; i += 64) acc[i] = (T)0;
        // octants in which a box of the pass has a child
        int pm = 0;
        if constexpr (BX == 16) {
            pm = 255;
        } else {
            const int bl = lane >> 3, o = lane & 7;
            int mk = 0;
            if constexpr (CMP) mk = __shfl(my_mask, (b0 + bl) & (kBoxTile - 1), 64);
            else mk = lane < BX * 8 && b0 + bl < kBoxTile ? smask[b0 + bl] : 0;
            const bool has = lane < BX * 8 && b0 + bl < kBoxTile && ((mk >> o) & 1);
            const unsigned long long bal = __ballot(has);
#pragma unroll
            for (int k = 0; k < BX; ++k) pm |= (int)((bal >> (8 * k)) & 255ull);
        }
        auto live = [&](int o) { return sfr[o] >= 0 && ((pm >> o) & 1); };
        int o0 = 0;
        while (o0 < 8) {
            // a chunk of whole octants with at most ME entries
            int o1 = o0 + 1;
            while (o1 < 8 && sgo[o1 + 1] - sgo[o0] <= ME) ++o1;
            const int e0 = sgo[o0], ne = sgo[o1] - e0;
            const int64_t eb = ebase + e0;
            wave_lds_fence();
            for (int i = lane; i < ne; i += 64) einfo[i] = Lc.te_info[eb + i];
            for (int i = lane; i < ne * BX; i += 64) {
                const int ei = i / BX, bl = i - ei * BX;
                const int bi = b0 + bl;
                int cs = bi < kBoxTile ? Lc.te_cs[(size_t)(eb + ei) * kBoxTile + bi] : -1;
                if (cs == -2) {
                    atomicAdd(kc.miss, (unsigned long long)((Lc.te_info[eb + ei] >> 8) & 255));
                    cs = -1;
                }
                ecs[i] = cs;
            }
            wave_lds_fence();
            // the frames of the chunk's live octants, one ahead in registers
            constexpr int RPL = (P + 63) / 64;
            T fq[RPL][5];
            int fo_ord[CMP ? RPL : 1];
            auto load_frame = [&](int o) {
                const int f = sfr[o];
#pragma unroll
                for (int h = 0; h < RPL; ++h) {
                    const int nu = lane + 64 * h;
                    const size_t e = (size_t)f * P + (nu < P ? nu : 0);
                    fq[h][0] = frt[3 * e];
                    fq[h][1] = frt[3 * e + 1];
                    fq[h][2] = frt[3 * e + 2];
                    fq[h][3] = frr[2 * e];
                    fq[h][4] = conj_sign * frr[2 * e + 1];
                    if constexpr (CMP) fo_ord[h] = Lc.fr_order[e];
                }
            };
            auto next_live = [&](int o) {
                while (o < o1 && !live(o)) ++o;
                return o;
            };
            int on = next_live(o0);
            if (on < o1) load_frame(on);
            while (on < o1) {
                const int o = on;
                // the octant's frame (loaded one octant ahead): coordinates and
                // ratio of every point
#pragma unroll
                for (int h = 0; h < RPL; ++h) {
                    const int nu = lane + 64 * h;
                    if (nu < P) {
                        rt[0][nu] = fq[h][0];
                        rt[1][nu] = fq[h][1];
                        rt[2][nu] = fq[h][2];
                        rg[0][nu] = fq[h][3];
                        rg[1][nu] = fq[h][4];
                        if constexpr (CMP) sord[nu] = (uint8_t)fo_ord[h];
                    }
                }
                on = next_live(o + 1);
                if (on < o1) load_frame(on);
                const int e_lo = sgo[o] - e0, e_hi = sgo[o + 1] - e0;
                if (e_lo < e_hi) fetch_b(e_lo);
                wave_lds_fence();
                const uint8_t* ord = &sord[CMP ? 0 : o * P];
                for (int ei = e_lo; ei < e_hi; ++ei) {
                    const int info = einfo[ei];
                    const int g0 = info & 255, cnt = (info >> 8) & 255;
                    // the first entry's operands were loaded with the frame
                    if (ei > e_lo) fetch_b(ei);
                    const T(&b)[NT][NK] = bn;
                    for (int t0 = 0; t0 < cnt; t0 += 16) {
                        const int rr = t0 + row;
                        const int nu_r = ord[g0 + (rr < cnt ? rr : 0)];
                        T Ls[PS], Lt[PA], Lpv[PA];
                        lagrange<T, PS>((double)rt[0][nu_r], kc.cs, Ls);
                        lagrange<T, PA>((double)rt[1][nu_r], kc.ca, Lt);
                        lagrange<T, PA>((double)rt[2][nu_r], kc.ca, Lpv);
                        if (rr >= cnt) {
#pragma unroll
                            for (int i = 0; i < PS; ++i) Ls[i] = (T)0;
                        }
                        mvec<T> c[NT];
                        mfma_tile<PS, PA, NT>(b, Ls, Lt, Lpv, q, c);
                        // the lane's rows: ratio times value into the pass's accumulators
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int ri = t0 + mfma_row<T>(q, i);
                            if constexpr (HALF) {
                                // the other part of the lane's complex column is in lane ^ 1
                                const T v = c[0][i];
                                const T pv = __shfl_xor(v, 1, 64);
                                if (ri < cnt) {
                                    const int nu = ord[g0 + ri];
                                    const T gr = rg[0][nu], gi = rg[1][nu];
                                    acc[nu * AS + col] += (col & 1) == 0 ? v * gr - pv * gi : pv * gi + v * gr;
                                }
                            } else {
                                if (ri < cnt) {
                                    const int nu = ord[g0 + ri];
                                    const T vr = c[0][i], vi = c[NT - 1][i];
                                    const T gr = rg[0][nu], gi = rg[1][nu];
                                    acc[aix(nu, col)] += vr * gr - vi * gi;
                                    acc[aix(nu, 16 + col)] += vr * gi + vi * gr;
                                }
                            }
                        }
                    }
                }
                wave_lds_fence();
            }
            o0 = o1;
        }
        wave_lds_fence();
        // write the pass's slots: column cc is (box cc / RB, right-hand side cc % RB)
        for (int i = lane; i < P * CP; i += 64) {
            const int nu = i / CP, cc = i - nu * CP;
            const int bl = cc / RB, r = cc - bl * RB;
            const int bi = b0 + bl;
            int sv = -1;
            if constexpr (CMP) sv = __shfl(my_slot, bi & (kBoxTile - 1), 64);
            else sv = bi < kBoxTile ? bslot[bi] : -1;
            const int s = bi < kBoxTile ? sv : -1;
            const int ir = HALF ? 2 * cc : cc, ii = HALF ? 2 * cc + 1 : 16 + cc;
            if (s >= 0) Fp[((size_t)s * P + nu) * RB + r] = cpx<T>{acc[aix(nu, ir)], acc[aix(nu, ii)]};
        }
        wave_lds_fence();
    }
}

// Interpolation at cousin targets for batched right-hand sides on the matrix
// cores (FP32), through the tabulated pairs.  One wavefront takes a target
// box and up to 16 of its targets as the rows of 16 x 16 x 4 MFMA tiles;
// for every cousin box, the rows whose targets fall into the same cone form
// one tile group: K = the cone's nodes (ordered as in mfma_tile), columns the
// real and imaginary parts of the RB right-hand sides, rows of other cones
// weighted zero.  Each row is multiplied by its centred factor G(x, x_k) and
// accumulated in registers, so a target's output is updated once, by one
// lane, after all cousins.
template <int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_eval_mfma(KernelConsts kc, LevelDev L,
                                                             const cpx<float>* __restrict__ F,
                                                             cpx<float>* __restrict__ out)
{
    constexpr int NC = 2 * RB;
    constexpr int NT = (NC + 15) / 16;
    constexpr int W = kBlock / 64;
    constexpr int NK = PS * PA + (PS * PA * (PA - 4) + 3) / 4;
    constexpr int P = PS * PA * PA;
    static_assert(PA >= 4, "the K ordering needs at least four phi nodes");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int tb = xcd_block(blockIdx.x, gridDim.x) * W + wv;
    if (tb >= L.nbox) return;                  // whole wavefront leaves
    const int row = lane & 15, q = lane >> 4, col = lane & 15;
    const int b0 = L.box_start[tb];
    const int nT = L.box_start[tb + 1] - b0;
    const long long base = L.pair_base[tb];
    const int nc = L.cou_start[tb + 1] - L.cou_start[tb];
    const long long np = L.npairs_cou;
    const float* pt = (const float*)L.pr_t;
    const float* pg = (const float*)L.pr_g;
    const float conj_sign = kc.adj ? -1.f : 1.f;
    const float* Ff = (const float*)F;
    float* outf = (float*)out;

    for (int r0 = 0; r0 < nT; r0 += 16) {
        const int tl = r0 + row;
        const bool valid = tl < nT;
        mf4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mf4{0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < nc; ++c) {
            const long long e = base + (long long)c * nT + (valid ? tl : 0);
            const int slot = valid ? L.pr_slot[e] : -1;
            if (valid && slot < 0 && q == 0) atomicAdd(kc.miss, 1ull);
            float Ls[PS], Lt[PA], Lpv[PA];
            lagrange<float, PS>((double)pt[e], kc.cs, Ls);
            lagrange<float, PA>((double)pt[np + e], kc.ca, Lt);
            lagrange<float, PA>((double)pt[2 * np + e], kc.ca, Lpv);
            const float gr = pg[e], gi = conj_sign * pg[np + e];
            // rows grouped by cone (lanes 0..15 hold one row each)
            unsigned long long todo = __ballot(lane < 16 && slot >= 0);
            while (todo) {
                const int leader = __ffsll((long long)todo) - 1;
                const int key = __shfl(slot, leader, 64);
                const bool in = slot == key;
                todo &= ~__ballot(lane < 16 && in);
                float Lsm[PS];
#pragma unroll
                for (int a = 0; a < PS; ++a) Lsm[a] = in ? Ls[a] : 0.f;
                float b[NT][NK];
                mfma_load_b<PS, PA, NC, NT>(Ff + (size_t)key * P * NC, q, col, b);
                mf4 cm[NT];
                mfma_tile<PS, PA, NT>(b, Lsm, Lt, Lpv, q, cm);
                // rows 4q + i: times the row's centred factor (columns 2m, 2m + 1: re, im)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float rgr = __shfl(gr, 4 * q + i, 64), rgi = __shfl(gi, 4 * q + i, 64);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const float v = cm[t][i];
                        const float pv = __shfl_xor(v, 1, 64);
                        acc[t][i] += (col & 1) == 0 ? v * rgr - pv * rgi : pv * rgi + v * rgr;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + 4 * q + i;
            if (r < nT) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int cg = 16 * t + col;
                    if (cg < NC) outf[((size_t)(b0 + r) * RB) * 2 + cg] += acc[t][i];
                }
            }
        }
    }
}

// Phase 1 for batched right-hand sides on the matrix cores: a wavefront
// takes 16 consecutive pairs in cone order as the rows of MFMA tiles; the
// rows that share a cone (usually all) form one tile group with that cone's
// values as the B operand (K = its nodes, columns the real and imaginary
// parts of the RB right-hand sides).  Each row is multiplied by its centred
// factor and stored once, at the pair's place.  FP32 uses 16 x 16 x 4 tiles;
// FP64 the 16 x 16 x 4 or, with at most 8 real columns, the four-block
// 4 x 4 x 4 instruction (the tiles of mfma_tile with CW columns).
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_pairs_values_mfma(KernelConsts kc, LevelDev L,
                                                                     const cpx<T>* __restrict__ F,
                                                                     cpx<T>* __restrict__ pval)
{
    constexpr int NC = 2 * RB;
    constexpr int CW = (sizeof(T) == 8 && NC <= 8) ? 4 : 16;
    constexpr int NT = (NC + CW - 1) / CW;
    constexpr int NO = CW == 16 ? 4 : 1;       // output elements per lane and tile
    constexpr int W = kBlock / 64;
    constexpr int NK = PS * PA + (PS * PA * (PA - 4) + 3) / 4;
    constexpr int P = PS * PA * PA;
    static_assert(PA >= 4, "the K ordering needs at least four phi nodes");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const long long no = L.npairs_ord;
    const long long i0 = ((long long)xcd_block(blockIdx.x, gridDim.x) * W + wv) * 16;
    if (i0 >= no) return;                      // whole wavefront leaves
    const int row = lane & 15, q = lane >> 4, col = lane % CW;
    const long long i = i0 + row;
    const bool valid = i < no;
    const long long ic = valid ? i : i0;
    const int slot = valid ? L.pro_slot[ic] : -1;
    const T* pt = (const T*)L.pro_t;
    const T* pg = (const T*)L.pro_g;
    T Ls[PS], Lt[PA], Lpv[PA];
    lagrange<T, PS>((double)pt[ic], kc.cs, Ls);
    lagrange<T, PA>((double)pt[no + ic], kc.ca, Lt);
    lagrange<T, PA>((double)pt[2 * no + ic], kc.ca, Lpv);
    const T gr = pg[ic], gi = (kc.adj ? (T)-1 : (T)1) * pg[no + ic];
    const long long e = L.pr_order[ic];       // -1: a placeholder, not stored
    const T* Ff = (const T*)F;
    T* pf = (T*)pval;
    unsigned long long todo = __ballot(lane < 16 && valid);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int key = __shfl(slot, leader, 64);
        const bool in = valid && slot == key;
        todo &= ~__ballot(lane < 16 && in);
        T Lsm[PS];
#pragma unroll
        for (int a = 0; a < PS; ++a) Lsm[a] = in ? Ls[a] : (T)0;
        T b[NT][NK];
        mfma_load_b<PS, PA, NC, NT, CW>(Ff + (size_t)key * P * NC, q, col, b);
        macc<T, CW> cm[NT];
        mfma_tile<PS, PA, NT, CW>(b, Lsm, Lt, Lpv, q, cm);
#pragma unroll
        for (int ii = 0; ii < NO; ++ii) {
            const int r = mfma_out_row<CW, T>(lane, ii);
            const T rgr = __shfl(gr, r, 64), rgi = __shfl(gi, r, 64);
            const int rin = __shfl((int)in, r, 64);
            const long long re = __shfl(e, r, 64);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                T v;
                if constexpr (CW == 16) v = cm[t][ii];
                else v = cm[t];
                const T pv = __shfl_xor(v, 1, 64);
                const int cg = CW * t + col;
                if (rin && re >= 0 && cg < NC)
                    pf[(size_t)re * NC + cg] = (col & 1) == 0 ? v * rgr - pv * rgi : pv * rgi + v * rgr;
            }
        }
    }
}

// Phase 1 for batched right-hand sides on levels without a pair table, on the
// matrix cores: the pairs in cone order (go_ord), 64 per wavefront.  Every
// lane takes one pair -- its target, its cousin, the pair's place in the
// value buffer, the cone holding the target, the target's local coordinates
// in it and G(x_t, x_c), all in FP64 as k_cousin_pairs_geo does -- and the
// wavefront then runs the pairs as four tiles of 16 rows, those of one cone
// (usually all) in one group with that cone's values as the B operand, as
// k_cousin_pairs_values_mfma does.  Each row's value times its factor is
// stored once, at the pair's place; phase 2 is k_cousin_pairs_sum_geo.
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1)))
k_cousin_pairs_go_mfma(KernelConsts kc, LevelDev L,
                                                                 const double* __restrict__ pts,
                                                                 const long long* __restrict__ pair_off,
                                                                 const uint32_t* __restrict__ ord, long long no,
                                                                 const cpx<T>* __restrict__ F,
                                                                 cpx<T>* __restrict__ pval)
{
    constexpr int NC = 2 * RB;
    constexpr int CW = (sizeof(T) == 8 && NC <= 8) ? 4 : 16;
    constexpr int NT = (NC + CW - 1) / CW;
    constexpr int NO = CW == 16 ? 4 : 1;       // output elements per lane and tile
    constexpr int W = kBlock / 64;
    constexpr int NK = PS * PA + (PS * PA * (PA - 4) + 3) / 4;
    constexpr int P = PS * PA * PA;
    static_assert(PA >= 4, "the K ordering needs at least four phi nodes");
    __shared__ int sslot[W][64];               // cone of each pair, -1: none
    __shared__ long long splace[W][64];        // its place in the value buffer
    __shared__ T stc[W][3][64];                // local coordinates
    __shared__ T sgr[W][64], sgi[W][64];       // G(x_t, x_c)
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const long long i0 = ((long long)xcd_block(blockIdx.x, gridDim.x) * W + wv) * 64;
    if (i0 >= no) return;                      // whole wavefront leaves
    T* pf = (T*)pval;
    {
        const long long i = i0 + lane;
        const uint32_t v = i < no ? ord[i] : 0xffffffffu;
        int slot = -1;
        long long place = -1;
        T t0 = (T)0, t1 = (T)0, t2 = (T)0, gr = (T)0, gi = (T)0;
        if (v != 0xffffffffu) {
            const int tp = (int)(v & 0xffffffu), ci = (int)(v >> 24);
            const int tb = L.pt_box[tp];
            const int b0 = L.box_start[tb];
            const int nT = L.box_start[tb + 1] - b0;
            const int c = L.cou[L.cou_start[tb] + ci];
            place = pair_off[tb] + (long long)ci * nT + (tp - b0);
            ConeLoc cl;
            cone_locate(pts[3 * tp] - L.box_ctr[3 * c], pts[3 * tp + 1] - L.box_ctr[3 * c + 1],
                        pts[3 * tp + 2] - L.box_ctr[3 * c + 2], L.h, L.ds, L.dang, L.ns, L.nc, cl);
            slot = lookup(L, c, cl.cell, cl.is);
            if (slot < 0) {
                // (the order holds only pairs whose cone the plan found)
                atomicAdd(kc.miss, 1ull);
                for (int r = 0; r < NC; ++r) pf[(size_t)place * NC + r] = (T)0;
                place = -1;
            } else {
                t0 = (T)cl.ts;
                t1 = (T)cl.tt;
                t2 = (T)cl.tp;
                T cs, sn;
                expi<T>(kc.kappa * cl.r, cs, sn);
                const T inv = (T)(kInv4Pi / cl.r);
                gr = cs * inv;
                gi = sn * inv;
            }
        }
        sslot[wv][lane] = slot;
        splace[wv][lane] = place;
        stc[wv][0][lane] = t0;
        stc[wv][1][lane] = t1;
        stc[wv][2][lane] = t2;
        sgr[wv][lane] = gr;
        sgi[wv][lane] = gi;
    }
    wave_lds_fence();
    const int row = lane & 15, q = lane >> 4, col = lane % CW;
    const T* Ff = (const T*)F;
    for (int r0 = 0; r0 < 64; r0 += 16) {
        const int rs = sslot[wv][r0 + row];
        T Ls[PS], Lt[PA], Lpv[PA];
        lagrange<T, PS>((double)stc[wv][0][r0 + row], kc.cs, Ls);
        lagrange<T, PA>((double)stc[wv][1][r0 + row], kc.ca, Lt);
        lagrange<T, PA>((double)stc[wv][2][r0 + row], kc.ca, Lpv);
        unsigned long long todo = __ballot(lane < 16 && rs >= 0);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const int key = __shfl(rs, leader, 64);
            const bool in = rs >= 0 && rs == key;
            todo &= ~__ballot(lane < 16 && in);
            T Lsm[PS];
#pragma unroll
            for (int a = 0; a < PS; ++a) Lsm[a] = in ? Ls[a] : (T)0;
            T b[NT][NK];
            mfma_load_b<PS, PA, NC, NT, CW>(Ff + (size_t)key * P * NC, q, col, b);
            macc<T, CW> cm[NT];
            mfma_tile<PS, PA, NT, CW>(b, Lsm, Lt, Lpv, q, cm);
#pragma unroll
            for (int ii = 0; ii < NO; ++ii) {
                const int r = r0 + mfma_out_row<CW, T>(lane, ii);
                const bool rin = sslot[wv][r] == key;
                const long long re = splace[wv][r];
                const T rgr = sgr[wv][r], rgi = sgi[wv][r];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    T v;
                    if constexpr (CW == 16) v = cm[t][ii];
                    else v = cm[t];
                    const T pv = __shfl_xor(v, 1, 64);
                    const int cg = CW * t + col;
                    if (rin && re >= 0 && cg < NC)
                        pf[(size_t)re * NC + cg] = (col & 1) == 0 ? v * rgr - pv * rgi : pv * rgi + v * rgr;
                }
            }
        }
    }
}

// ----------------------------------------------------------- gradients

// d/dx of the near field: sum_j a_j G(x, x_j) (i k - 1/r) (x - x_j) / r,
// contracted with conj(g): grad[i][c] = sum_r Re(conj(g_r) dI_r/dx_c).
template <typename T, int RB>
__global__ void __launch_bounds__(kBlock) k_near_grad(KernelConsts kc, LevelDev L, const double* __restrict__ pts,
                                                      const cpx<T>* __restrict__ dens, const cpx<T>* __restrict__ gout,
                                                      double* __restrict__ grad)
{
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int b = L.pt_box[i];
    const double x0 = pts[3 * i], x1 = pts[3 * i + 1], x2 = pts[3 * i + 2];
    cpx<T> g[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) g[r] = gout[(size_t)i * RB + r];
    double acc0 = 0, acc1 = 0, acc2 = 0;
    const int e1 = near_end(L, b);
    for (int e = near_first(L, b); e < e1; ++e) {
        int lo, hi;
        near_range(L, e, lo, hi);
        for (int j = lo; j < hi; ++j) {
            if (j == i) continue;
            double dx = x0 - pts[3 * j], dy = x1 - pts[3 * j + 1], dz = x2 - pts[3 * j + 2];
            double rr = sqrt(dx * dx + dy * dy + dz * dz);
            T c, s;
            expi<T>(kc.kappa * rr, c, s);
            T inv = (T)(kInv4Pi / rr);
            // G (i k - 1/r) / r
            T gr = c * inv, gi = s * inv;
            T fr = (T)(-1.0 / rr), fi = (T)kc.kappa;
            T hr = (gr * fr - gi * fi) * (T)(1.0 / rr), hi = (gr * fi + gi * fr) * (T)(1.0 / rr);
            // s = sum_r Re(conj(g_r) a_r h)
            T sr = (T)0;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                cpx<T> a = dens[(size_t)j * RB + r];
                T ar = a.x * hr - a.y * hi, ai = a.x * hi + a.y * hr;
                sr += g[r].x * ar + g[r].y * ai;
            }
            acc0 += (double)sr * dx;
            acc1 += (double)sr * dy;
            acc2 += (double)sr * dz;
        }
    }
    grad[3 * i] = acc0;
    grad[3 * i + 1] = acc1;
    grad[3 * i + 2] = acc2;
}

// d/dx of the cousin-target interpolation at level d:
//   d/dx [G(x, x_k) P] = P grad G + G (dP/dts 2/ds grad s + dP/dtt 2/dang grad theta
//                                      + dP/dtp 2/dang grad phi),
// grad s = -s v / r^2, grad theta = (vx vz, vy vz, -rho^2) / (rho r^2),
// grad phi = (-vy, vx, 0) / rho^2 (rho > 0; on the polar axis see below).
template <typename T, int PS, int PA, int RB>
__global__ void __launch_bounds__(kBlock) k_cousin_grad(KernelConsts kc, LevelDev L, const double* __restrict__ pts,
                                                        const cpx<T>* __restrict__ F, const cpx<T>* __restrict__ gout,
                                                        double* __restrict__ grad)
{
    const int P = PS > 0 ? PS * PA * PA : kc.ps * kc.pa * kc.pa;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= kc.n) return;
    const int t = L.pt_box[i];
    const double x0 = pts[3 * i], x1 = pts[3 * i + 1], x2 = pts[3 * i + 2];
    cpx<T> g[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) g[r] = gout[(size_t)i * RB + r];
    double acc0 = 0, acc1 = 0, acc2 = 0;
    for (int ci = L.cou_start[t]; ci < L.cou_start[t + 1]; ++ci) {
        const int k = L.cou[ci];
        const double v0 = x0 - L.box_ctr[3 * k], v1 = x1 - L.box_ctr[3 * k + 1], v2 = x2 - L.box_ctr[3 * k + 2];
        ConeLoc cl;
        cone_locate(v0, v1, v2, L.h, L.ds, L.dang, L.ns, L.nc, cl);
        const int slot = lookup(L, k, cl.cell, cl.is);
        if (slot < 0) {
            atomicAdd(kc.miss, 1ull);
            continue;
        }
        constexpr int NS = basis_len<PS>(), NA = basis_len<PA>();
        T Ls[NS], Lt[NA], Lp[NA], dLs[NS], dLt[NA], dLp[NA];
        basis_d<T, PS>(cl.ts, kc.cs, kc.ps, Ls, dLs);
        basis_d<T, PA>(cl.tt, kc.ca, kc.pa, Lt, dLt);
        basis_d<T, PA>(cl.tp, kc.ca, kc.pa, Lp, dLp);
        cpx<T> v[RB], vs[RB], vt[RB], vp[RB];
        interp_n<T, PS, PA, RB>(F + (size_t)slot * P * RB, Ls, Lt, Lp, kc, v);
        interp_n<T, PS, PA, RB>(F + (size_t)slot * P * RB, dLs, Lt, Lp, kc, vs);
        interp_n<T, PS, PA, RB>(F + (size_t)slot * P * RB, Ls, dLt, Lp, kc, vt);
        interp_n<T, PS, PA, RB>(F + (size_t)slot * P * RB, Ls, Lt, dLp, kc, vp);
        const double r = cl.r, r2 = r * r;
        const double rho2 = v0 * v0 + v1 * v1, rho = sqrt(rho2);
        const double cs_ = 2.0 / L.ds, ca_ = 2.0 / L.dang;
        const double gs[3] = {-cl.s * v0 / r2 * cs_, -cl.s * v1 / r2 * cs_, -cl.s * v2 / r2 * cs_};
        double gt[3], gp[3];
        if (rho > 0.0) {
            gt[0] = v0 * v2 / (rho * r2) * ca_;
            gt[1] = v1 * v2 / (rho * r2) * ca_;
            gt[2] = -rho / r2 * ca_;
            gp[0] = -v1 / rho2 * ca_;
            gp[1] = v0 / rho2 * ca_;
            gp[2] = 0.0;
        } else {
            // on the frame's polar axis phi is undefined and the interpolant is
            // not differentiable across the axis: take the derivative along it
            // plus the one-sided derivative into the half-plane phi = 0 that
            // holds the axis (atan2(0, 0) = 0): grad theta = (cos theta, 0, 0) / r,
            // no phi term
            gt[0] = v2 / r2 * ca_;
            gt[1] = gt[2] = 0.0;
            gp[0] = gp[1] = gp[2] = 0.0;
        }
        T c, s;
        expi<T>(kc.kappa * r, c, s);
        T inv = (T)(kInv4Pi / r);
        T Gr = c * inv, Gi = s * inv;
        // grad G = G (i k - 1/r) v / r
        T fr = (T)(-1.0 / r), fi = (T)kc.kappa;
        T Hr = (Gr * fr - Gi * fi) * (T)(1.0 / r), Hi = (Gr * fi + Gi * fr) * (T)(1.0 / r);
        // per RHS: Re(conj(g) (P H v_c + G (Ps gs_c + Pt gt_c + Pp gp_c)))
        double sP = 0, sS = 0, sT = 0, sPh = 0;
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            T pr = v[rr].x * Hr - v[rr].y * Hi, pi = v[rr].x * Hi + v[rr].y * Hr;           // P H
            sP += (double)(g[rr].x * pr + g[rr].y * pi);
            T qr = vs[rr].x * Gr - vs[rr].y * Gi, qi = vs[rr].x * Gi + vs[rr].y * Gr;       // Ps G
            sS += (double)(g[rr].x * qr + g[rr].y * qi);
            qr = vt[rr].x * Gr - vt[rr].y * Gi;
            qi = vt[rr].x * Gi + vt[rr].y * Gr;
            sT += (double)(g[rr].x * qr + g[rr].y * qi);
            qr = vp[rr].x * Gr - vp[rr].y * Gi;
            qi = vp[rr].x * Gi + vp[rr].y * Gr;
            sPh += (double)(g[rr].x * qr + g[rr].y * qi);
        }
        acc0 += sP * v0 + sS * gs[0] + sT * gt[0] + sPh * gp[0];
        acc1 += sP * v1 + sS * gs[1] + sT * gt[1] + sPh * gp[1];
        acc2 += sP * v2 + sS * gs[2] + sT * gt[2] + sPh * gp[2];
    }
    grad[3 * i] += acc0;
    grad[3 * i + 1] += acc1;
    grad[3 * i + 2] += acc2;
}

// [n][3] (Morton order) -> grad [wn][3], the window's points (input order);
// with acc the values are added (passes of right-hand sides after the first).
__global__ void __launch_bounds__(kBlock) k_permute_grad(const double* __restrict__ in, double* __restrict__ out,
                                                         const int32_t* __restrict__ iperm, Window w, int acc)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= w.wn) return;
    int i = iperm[w.w0 + j];
    if (acc) {
        out[3 * j] += in[3 * i];
        out[3 * j + 1] += in[3 * i + 1];
        out[3 * j + 2] += in[3 * i + 2];
    } else {
        out[3 * j] = in[3 * i];
        out[3 * j + 1] = in[3 * i + 1];
        out[3 * j + 2] = in[3 * i + 2];
    }
}

// ------------------------------------------------------------- host side

// Blocks of kBlock threads for `items` threads.  A dispatch counts its
// work-items in 32 bits, so a launch of 2^32 or more would be cut short:
// such a request gives 0 blocks, and the launch fails (IFGF_E_HIP) instead of
// silently covering part of the items.
inline unsigned grid_for(size_t items)
{
    const size_t b = (items + kBlock - 1) / kBlock;
    return b * kBlock >= ((size_t)1 << 32) ? 0u : (unsigned)b;
}

// Source and target windows of a plan: every point is both unless the plan
// was created with distinct targets.
inline Window source_window(const DevicePlan& p)
{
    return p.n_tgt > 0 ? Window{0, (int)p.n_src} : Window{0, (int)p.hp.n};
}
inline Window target_window(const DevicePlan& p)
{
    return p.n_tgt > 0 ? Window{(int)p.n_src, (int)p.n_tgt} : Window{0, (int)p.hp.n};
}

inline int rb_for(int nrhs) { return nrhs >= 5 ? 16 : (nrhs >= 2 ? 4 : 1); }

// Pairs the per-pair value buffer holds: those of the largest tabulated level,
// and of the largest untabulated one when that fits the budget
// (IFGF_PVAL_BUDGET_MB, default 32768) at rb right-hand sides.
}  // namespace

// Waits for the plan's work on every stream that ran it (its callers'
// streams, its side and capture streams), not for the whole device.
hipError_t wait_plan_streams(DevicePlan& p)
{
    hipError_t e = hipSuccess;
    for (hipStream_t u : p.used_streams)
        if (e == hipSuccess) e = hipStreamSynchronize(u);
    if (e == hipSuccess && p.side) e = hipStreamSynchronize(p.side);
    if (e == hipSuccess && p.cap_stream) e = hipStreamSynchronize(p.cap_stream);
    if (e == hipSuccess) {
        // keep only the latest caller stream: the others have drained
        p.used_streams.clear();
        p.used_streams.push_back(p.last_stream);
    }
    return e;
}

namespace {

inline bool compiled_degrees(int ps, int pa) { return (ps == 3 && pa == 5) || (ps == 4 && pa == 6) || (ps == 2 && pa == 3); }

inline int64_t pval_pairs_for(const DevicePlan& p, int rb, size_t ce)
{
    // the kernels for run-time node counts evaluate cousins in one pass
    if (!compiled_degrees(p.hp.ps, p.hp.pang)) return 0;
    int64_t geo = 0;
    for (int d = 3; d <= p.hp.D; ++d)
        if (!p.hp.L[d].use_pairs) geo = std::max<int64_t>(geo, p.npairs_all[d]);
    const char* v = std::getenv("IFGF_PVAL_BUDGET_MB");
    const double budget = (v && *v ? std::atof(v) : 32768.0) * 1024.0 * 1024.0;
    if ((double)geo * rb * ce > budget) geo = 0;
    return std::max<int64_t>(p.max_pairs, geo);
}

// Workspaces for `rb` right-hand sides per pass; cone values either for every
// level (store) or in two buffers used alternately.  Sets *fresh when the
// buffers were (re)allocated, which discards stored cone values.
template <typename T>
hipError_t ensure_workspace(DevicePlan& p, int rb, bool store, bool* fresh)
{
    const HostPlan& hp = p.hp;
    const int D = hp.D;
    if (fresh) *fresh = false;
    if (p.ws_rb >= rb && p.ws_store == store) return hipSuccess;
    if (fresh) *fresh = true;
    // the old buffers may still be read by earlier calls' kernels
    hipError_t e = wait_plan_streams(p);
    if (e != hipSuccess) return e;
    for (void* q : p.ws_allocs) (void)hipFree(q);
    p.ws_allocs.clear();
    p.ws_bytes = 0;
    p.ws_rb = 0;
    p.dens_m = p.out_m = p.gout_m = nullptr;
    p.grad_m = nullptr;
    for (auto& f : p.F) f = nullptr;
    p.stored_valid = false;
    const size_t ce = sizeof(cpx<T>);
    size_t need = 3 * (size_t)hp.n * rb * ce + (size_t)hp.n * 3 * sizeof(double);
    size_t maxs = 0, tot = 0;
    for (int d = 3; d <= D; ++d) {
        maxs = std::max(maxs, (size_t)hp.L[d].nslots);
        tot += (size_t)hp.L[d].nslots;
    }
    const int64_t pv_pairs = pval_pairs_for(p, rb, ce);
    need += (store ? tot : 2 * maxs) * hp.P * rb * ce + (size_t)pv_pairs * rb * ce;
    if (p.ws_limit && p.tree_bytes + need > p.ws_limit) return hipErrorOutOfMemory;
    auto alloc = [&](size_t bytes, void** out) -> hipError_t {
        if (bytes == 0) bytes = 16;
        hipError_t err = hipMalloc(out, bytes);
        if (err == hipSuccess) {
            p.ws_allocs.push_back(*out);
            p.ws_bytes += bytes;
        }
        return err;
    };
    if ((e = alloc((size_t)hp.n * rb * ce, &p.dens_m)) != hipSuccess) return e;
    if ((e = alloc((size_t)hp.n * rb * ce, &p.out_m)) != hipSuccess) return e;
    if ((e = alloc((size_t)hp.n * rb * ce, &p.gout_m)) != hipSuccess) return e;
    void* gm = nullptr;
    if ((e = alloc((size_t)hp.n * 3 * sizeof(double), &gm)) != hipSuccess) return e;
    p.grad_m = (double*)gm;
    p.pval = nullptr;
    p.pval_pairs = 0;
    if (pv_pairs > 0 && (e = alloc((size_t)pv_pairs * rb * ce, &p.pval)) != hipSuccess) return e;
    p.pval_pairs = pv_pairs;
    if (store) {
        for (int d = 3; d <= D; ++d)
            if ((e = alloc((size_t)hp.L[d].nslots * hp.P * rb * ce, &p.F[d])) != hipSuccess) return e;
    } else if (D >= 3) {
        void* buf[2];
        if ((e = alloc(maxs * hp.P * rb * ce, &buf[0])) != hipSuccess) return e;
        if ((e = alloc(maxs * hp.P * rb * ce, &buf[1])) != hipSuccess) return e;
        for (int d = 3; d <= D; ++d) p.F[d] = buf[d & 1];
    }
    p.ws_rb = rb;
    p.ws_store = store;
    ++p.ws_gen;
    return hipSuccess;
}

// Entries (octant, child-cone group) per box tile from which the default
// takes the half-width box kernel: 16 in FP64, 20 in FP32 (4 RHS).
template <typename T>
constexpr double half_entries()
{
    return std::is_same<T, double>::value ? 16.0 : 20.0;
}

// FP64 box kernel in its compact LDS layout (seven wavefronts per CU) on the
// levels whose frames allow it (IFGF_BOXACC_COMPACT=0: never).
inline bool boxacc_compact()
{
    const char* v = std::getenv("IFGF_BOXACC_COMPACT");
    return !(v && *v && std::atoi(v) == 0);
}

// Least average number of slots per box tile (as a fraction of kBoxTile) for
// which the default rule picks the box-batched child-to-parent kernel (never
// for 16 right-hand sides, where the autotuner decides); IFGF_BOX_FILL
// overrides it (a value above 1 disables it in the default rule).
inline double box_fill_min(int rb)
{
    const char* v = std::getenv("IFGF_BOX_FILL");
    if (v && *v) return std::atof(v);
    return rb == 1 ? 0.5 : (rb == 4 ? 0.25 : 2.0);
}

// Child-to-parent kernel variants of level d (children at d).  Every
// variant writes every parent slot, so any one of them can serve a level.
template <typename T, int PS, int PA, int RB>
int c2p_candidates(const DevicePlan& p, int d, int* v)
{
    if constexpr (PS == 0) {
        // run-time node counts: the geometry kernel only
        (void)p;
        (void)d;
        v[0] = kC2PGeometry;
        return 1;
    } else {
        constexpr int P = PS * PA * PA;
        constexpr int S = lds_slots<P, RB>();
        constexpr int GCAP = lds_gcap<T, P, RB, S>();
        const LevelDev& L = p.L[d];
        const bool groups = L.use_frames && L.frame_groups_ok;
        int n = 0;
        v[n++] = kC2PGeometry;
        if (L.use_frames) v[n++] = kC2PFrames;
        if constexpr (GCAP >= S) {
            if (groups) v[n++] = kC2PLds;
            if (groups && L.slot_order) v[n++] = kC2PLdsTiled;
        }
        if constexpr (RB >= 4 && PA >= 4 && P <= 128) {
            v[n++] = groups ? kC2PMfma : kC2PMfmaGeometry;
        }
        if constexpr (std::is_same<T, float>::value && PA >= 4 && P <= 128) {
            if (groups && L.ntiles > 0 && L.te_start) v[n++] = kC2PBoxes;
        }
        if constexpr (PA >= 4 && P <= 128) {
            if (groups && L.ntiles > 0 && L.te_start) v[n++] = kC2PBoxAcc;
        }
        if constexpr (RB <= 8 && PA >= 4 && P <= 128) {
            if (groups && L.ntiles > 0 && L.te_start) v[n++] = kC2PBoxAccHalf;
        }
        if constexpr (RB == 1 && P <= 255) {
            if (groups) v[n++] = kC2PQuads;
        }
        return n;
    }
}

// The variant used when the plan has not been tuned: the box-batched kernel
// where its tiles are full enough, else the matrix-core kernel for batched
// FP32, else LDS staging, else the frame or geometry kernel.
template <typename T, int PS, int PA, int RB>
int c2p_default(const DevicePlan& p, int d)
{
    if constexpr (PS == 0) {
        (void)p;
        (void)d;
        return kC2PGeometry;
    } else {
        int v[kC2PVariants];
        const int n = c2p_candidates<T, PS, PA, RB>(p, d, v);
        auto has = [&](int x) {
            for (int i = 0; i < n; ++i)
                if (v[i] == x) return true;
            return false;
        };
        const bool full = (double)p.hp.L[d - 1].nslots >= box_fill_min(RB) * kBoxTile * (double)p.L[d].ntiles;
        // with batched right-hand sides (and always in FP64) the kernel with
        // the accumulators in LDS measured faster; at 1 RHS in FP32 the one
        // with register accumulators
        // tiles with many entries (small child-cone groups) measured faster at
        // half width (more wavefronts per CU hide the operand loads)
        if (has(kC2PBoxAccHalf) && full && p.hp.L[d].te_per_tile >= half_entries<T>() &&
            (std::is_same<T, double>::value || RB >= 4))
            return kC2PBoxAccHalf;
        if (has(kC2PBoxAcc) && full && (std::is_same<T, double>::value || RB >= 4)) return kC2PBoxAcc;
        if (has(kC2PBoxes) && full) return kC2PBoxes;
        if (has(kC2PMfma)) return kC2PMfma;
        if (has(kC2PMfmaGeometry)) return kC2PMfmaGeometry;
        if (has(kC2PLds)) return kC2PLds;
        if (has(kC2PFrames)) return kC2PFrames;
        return kC2PGeometry;
    }
}

inline int rb_index(int rb) { return rb == 1 ? 0 : (rb == 4 ? 1 : 2); }

// Node counts served by the kernels instantiated for run-time node counts
// (PS = PA = 0): any other pair with 1 <= P_s, P_ang <= kMaxNodes.
inline bool any_degrees(int ps, int pa) { return ps >= 1 && ps <= kMaxNodes && pa >= 1 && pa <= kMaxNodes; }


template <typename T, int PS, int PA, int RB>
int c2p_variant(const DevicePlan& p, int d)
{
    const int c = p.c2p_choice[rb_index(RB)][d];
    return c >= 0 ? c : c2p_default<T, PS, PA, RB>(p, d);
}

template <typename T, int PS, int PA, int RB>
void c2p_launch(DevicePlan& p, const KernelConsts& kc, int d, int variant, hipStream_t st)
{
    if constexpr (PS == 0) {
        // run-time node counts: geometry computed per evaluation
        (void)variant;
        const int64_t nps = p.hp.L[d - 1].nslots;
        k_child_to_parent<T, 0, 0, RB><<<grid_for((size_t)nps * p.hp.P), kBlock, 0, st>>>(
            kc, p.L[d], p.L[d - 1], (const cpx<T>*)p.F[d], (cpx<T>*)p.F[d - 1]);
    } else {
        constexpr int P = PS * PA * PA;
        constexpr int S = lds_slots<P, RB>();
        constexpr int GCAP = lds_gcap<T, P, RB, S>();
        constexpr int NT = lds_threads<P, RB>();
        using C = cpx<T>;
        const int64_t nps = p.hp.L[d - 1].nslots;
        const C* Fc = (const C*)p.F[d];
        C* Fp = (C*)p.F[d - 1];
        switch (variant) {
        case kC2PBoxes:
            if constexpr (std::is_same<T, float>::value && PA >= 4 && P <= 128) {
                k_child_to_parent_boxes<PS, PA, RB><<<(unsigned)p.L[d].ntiles, 64, 0, st>>>(
                    kc, p.L[d], p.L[d - 1], Fc, Fp, (const C*)p.zero_cone);
                return;
            }
            break;
        case kC2PBoxAcc:
            if constexpr (PA >= 4 && P <= 128) {
                if constexpr (std::is_same<T, double>::value) {
                    if (p.hp.L[d].fr_max_groups <= kCompactEnt && boxacc_compact()) {
                        k_child_to_parent_boxacc<T, PS, PA, RB, false, true><<<(unsigned)p.L[d].ntiles, 64, 0, st>>>(
                            kc, p.L[d], p.L[d - 1], Fc, Fp, (const C*)p.zero_cone);
                        return;
                    }
                }
                k_child_to_parent_boxacc<T, PS, PA, RB, false><<<(unsigned)p.L[d].ntiles, 64, 0, st>>>(
                    kc, p.L[d], p.L[d - 1], Fc, Fp, (const C*)p.zero_cone);
                return;
            }
            break;
        case kC2PBoxAccHalf:
            if constexpr (RB <= 8 && PA >= 4 && P <= 128) {
                k_child_to_parent_boxacc<T, PS, PA, RB, true><<<(unsigned)p.L[d].ntiles, 64, 0, st>>>(
                    kc, p.L[d], p.L[d - 1], Fc, Fp, (const C*)p.zero_cone);
                return;
            }
            break;
        case kC2PMfma:
        case kC2PMfmaGeometry:
            if constexpr (RB >= 4 && PA >= 4 && P <= 128) {
                // wavefronts per block: the slots' accumulators in LDS stay under
                // about 40 KB per block
                constexpr int W = mfma_waves<T, P, RB>();
                const unsigned nb = (unsigned)((nps + W - 1) / W);
                if (variant == kC2PMfma)
                    k_child_to_parent_mfma<T, PS, PA, RB, W><<<nb, 64 * W, 0, st>>>(kc, p.L[d], p.L[d - 1], Fc, Fp);
                else
                    k_child_to_parent_mfma_geo<T, PS, PA, RB, W><<<nb, 64 * W, 0, st>>>(kc, p.L[d], p.L[d - 1], Fc, Fp);
                return;
            }
            break;
        case kC2PLds:
            if constexpr (GCAP >= S) {
                k_child_to_parent_lds<T, PS, PA, RB, S, GCAP, false, NT>
                    <<<(unsigned)((nps + S - 1) / S), NT, 0, st>>>(kc, p.L[d], p.L[d - 1], Fc, Fp);
                return;
            }
            break;
        case kC2PLdsTiled:
            if constexpr (GCAP >= S) {
                k_child_to_parent_lds<T, PS, PA, RB, S, GCAP, true, NT>
                    <<<(unsigned)((nps + S - 1) / S), NT, 0, st>>>(kc, p.L[d], p.L[d - 1], Fc, Fp);
                return;
            }
            break;
        case kC2PFrames:
            k_child_to_parent_frames<T, PS, PA, RB><<<grid_for((size_t)nps * P), kBlock, 0, st>>>(kc, p.L[d], p.L[d - 1],
                                                                                                 Fc, Fp);
            return;
        case kC2PQuads:
            if constexpr (RB == 1 && P <= 255) {
                constexpr int QS = kQuadSlots;
                constexpr int QR = std::is_same<T, float>::value ? 4 : 2;
                constexpr int QG = quad_gcap<T, P>();
                k_child_to_parent_quads<T, PS, PA, QS, QR, QG>
                    <<<(unsigned)((nps + QS - 1) / QS), kBlock, 0, st>>>(kc, p.L[d], p.L[d - 1], Fc, Fp);
                return;
            }
            break;
        default:
            break;
        }
        k_child_to_parent<T, PS, PA, RB><<<grid_for((size_t)nps * P), kBlock, 0, st>>>(kc, p.L[d], p.L[d - 1], Fc, Fp);
    }
}

// The matrix-core cousin evaluation for batched right-hand sides runs only
// with IFGF_COUSIN_MFMA=1: one target box per wavefront leaves it bound by
// the latency of its sequential cousin loop (3.7x slower than the vector
// kernel, which serves about ten boxes per wavefront, on the sphere
// N = 393216 with 16 right-hand sides).
inline bool cousin_mfma_enabled()
{
    const char* v = std::getenv("IFGF_COUSIN_MFMA");
    return v && *v && std::atoi(v) != 0;
}

// Two-phase cousin evaluation with one thread per pair (through the pair
// table where a level has one without a cone-ordered copy, else with the
// geometry per pair): on unless IFGF_COUSIN_GEO_PAIRS=0.
inline bool cousin_geo_pairs_enabled()
{
    const char* v = std::getenv("IFGF_COUSIN_GEO_PAIRS");
    return !(v && *v && std::atoi(v) == 0);
}

// Cousin pairs of levels without a pair table in cone order on the matrix
// cores (batched right-hand sides): on unless IFGF_COUSIN_GEO_ORDER=0.
inline bool cousin_geo_order_enabled()
{
    const char* v = std::getenv("IFGF_COUSIN_GEO_ORDER");
    return !(v && *v && std::atoi(v) == 0);
}

// Two-phase cousin evaluation for one right-hand side: on unless
// IFGF_COUSIN_TWO_PHASE=0.
inline bool cousin_two_phase_enabled()
{
    const char* v = std::getenv("IFGF_COUSIN_TWO_PHASE");
    return !(v && *v && std::atoi(v) == 0);
}

// IFGF_AUTOTUNE_VERBOSE=1: the autotuner prints every timing to stderr.
inline bool autotune_verbose()
{
    const char* v = std::getenv("IFGF_AUTOTUNE_VERBOSE");
    return v && *v && std::atoi(v) != 0;
}

// The second stream of an eager apply (IFGF_SIDE_STREAM=0: one stream).
inline bool side_stream_enabled()
{
    const char* v = std::getenv("IFGF_SIDE_STREAM");
    return !(v && *v && std::atoi(v) == 0);
}

// Creates the side stream (default priority) and its events once.
inline hipError_t ensure_side(DevicePlan& p)
{
    hipError_t e;
    if (!p.side && (e = hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking)) != hipSuccess) return e;
    const size_t need = 2 + 2 * (IFGF_MAX_LEVELS + 1);
    while (p.sync_ev.size() < need) {
        hipEvent_t ev;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
        p.sync_ev.push_back(ev);
    }
    return hipSuccess;
}

// Events of the two-stream apply: cone values of level d ready (main
// stream), and level d's cousin evaluation done (side stream).
inline hipEvent_t ev_ready(DevicePlan& p, int d) { return p.sync_ev[2 + d]; }
inline hipEvent_t ev_read(DevicePlan& p, int d) { return p.sync_ev[2 + IFGF_MAX_LEVELS + 1 + d]; }

// The cousin-target interpolation of level d (Algorithm 1, first inner
// loop) on stream st, or its gradient.
template <typename T, int PS, int PA, int RB>
void cousin_stage(DevicePlan& p, const KernelConsts& kc, int d, bool grad, hipStream_t st)
{
    const HostPlan& hp = p.hp;
    const int n = (int)hp.n;
    using C = cpx<T>;
    // nothing to interpolate: no source box of this level has cones, or no
    // target has a cousin that is a source box (an adaptive octree can leave
    // whole levels without source boxes)
    if (hp.L[d].nslots == 0 || p.npairs_all[d] == 0) return;
    if (grad) {
        StageTimer tm_(p, IFGF_STAGE_COUSIN_GRAD, st, d);
        k_cousin_grad<T, PS, PA, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], p.pts, (const C*)p.F[d],
                                                                     (const C*)p.gout_m, p.grad_m);
        return;
    }
    StageTimer tm_(p, IFGF_STAGE_COUSIN_EVAL, st, d);
    if constexpr (PS == 0) {
        // run-time node counts: one kernel, geometry computed per evaluation
        k_cousin_eval<T, 0, 0, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], p.pts, (const C*)p.F[d], (C*)p.out_m);
        return;
    } else {
        bool done = false;
        if constexpr (std::is_same<T, float>::value && RB >= 4 && PA >= 4) {
            if (p.L[d].use_pairs && cousin_mfma_enabled()) {
                k_cousin_eval_mfma<PS, PA, RB><<<(unsigned)((hp.L[d].nbox + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0,
                                                 st>>>(kc, p.L[d], (const C*)p.F[d], (C*)p.out_m);
                done = true;
            }
        }
        if (!done && p.L[d].use_pairs && p.L[d].npairs_ord > 0 && p.pval && cousin_two_phase_enabled()) {
            if constexpr (RB == 1) {
                k_cousin_pairs_values<T, PS, PA><<<grid_for((size_t)p.L[d].npairs_ord / kPairQuad), kBlock, 0, st>>>(
                    kc, p.L[d], (const C*)p.F[d], (C*)p.pval);
                done = true;
            } else if constexpr (PA >= 4) {
                const size_t waves = ((size_t)p.L[d].npairs_ord + 15) / 16;
                k_cousin_pairs_values_mfma<T, PS, PA, RB><<<(unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64)),
                                                            kBlock, 0, st>>>(kc, p.L[d], (const C*)p.F[d], (C*)p.pval);
                done = true;
            }
            if (done)
                k_cousin_pairs_sum<T, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], (const C*)p.pval, (C*)p.out_m);
        }
        if constexpr (RB >= 4 && PA >= 4) {
            // the pairs in cone order on the matrix cores, geometry per pair
            // (levels without a cone-ordered pair table)
            if (!done && p.go_ord[d] && p.pval && p.pair_off[d] && p.npairs_all[d] <= p.pval_pairs &&
                cousin_geo_pairs_enabled() && cousin_geo_order_enabled()) {
                const size_t waves = ((size_t)p.ngo[d] + 63) / 64;
                k_cousin_pairs_go_mfma<T, PS, PA, RB><<<(unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64)), kBlock,
                                                        0, st>>>(kc, p.L[d], p.pts, p.pair_off[d], p.go_ord[d],
                                                                 p.ngo[d], (const C*)p.F[d], (C*)p.pval);
                k_cousin_pairs_sum_geo<T, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], p.pair_off[d],
                                                                              (const C*)p.pval, (C*)p.out_m);
                done = true;
            }
        }
        if (done) {
        } else if (p.L[d].use_pairs && p.pval && p.L[d].npairs_cou <= p.pval_pairs && cousin_geo_pairs_enabled() &&
                   hp.n < 64 * (int64_t)hp.L[d].nbox) {
            // two phases through the pair table, where boxes hold few targets (in
            // large boxes the threads of one target box already walk the same
            // cousins together, and the one-kernel form measured faster)
            k_cousin_pairs_tab<T, PS, PA, RB><<<grid_for((size_t)p.L[d].npairs_cou), kBlock, 0, st>>>(
                kc, p.L[d], (const C*)p.F[d], (C*)p.pval);
            k_cousin_pairs_sum<T, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], (const C*)p.pval, (C*)p.out_m);
        } else if (p.L[d].use_pairs) {
            k_cousin_eval_pairs<T, PS, PA, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], (const C*)p.F[d],
                                                                               (C*)p.out_m);
        } else if (p.pval && p.pair_off[d] && p.npairs_all[d] <= p.pval_pairs && cousin_geo_pairs_enabled()) {
            // two phases with the geometry computed per pair, one thread per pair
            k_cousin_pairs_geo<T, PS, PA, RB><<<grid_for((size_t)p.npairs_all[d]), kBlock, 0, st>>>(
                kc, p.L[d], p.pts, p.pair_off[d], p.npairs_all[d], (const C*)p.F[d], (C*)p.pval);
            k_cousin_pairs_sum_geo<T, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], p.pair_off[d], (const C*)p.pval,
                                                                          (C*)p.out_m);
        } else {
            k_cousin_eval<T, PS, PA, RB><<<grid_for(n), kBlock, 0, st>>>(kc, p.L[d], p.pts, (const C*)p.F[d],
                                                                         (C*)p.out_m);
        }
    }
}

// Leaf values, then for d = D..3 the cousin evaluation of level d and the
// child-to-parent step d -> d - 1 (Algorithm 1).  With a side stream sd
// distinct from st, the cousin evaluations run on sd: level d's waits for
// its cone values, and a child-to-parent step whose output buffer held
// level d + 1 (ping-pong buffers) waits for that level's cousin evaluation.
// The caller joins sd back into st.
template <typename T, int PS, int PA, int RB>
hipError_t upward_and_eval(DevicePlan& p, const KernelConsts& kc, hipStream_t st, bool grad, bool reuse,
                           hipStream_t sd = nullptr)
{
    const HostPlan& hp = p.hp;
    const int D = hp.D;
    const int P = hp.P;
    using C = cpx<T>;
    const bool two = sd && sd != st;
    if (!sd) sd = st;
    if (D < 3) return hipSuccess;
    if (!reuse && hp.L[D].nslots > 0)
        {
            StageTimer tm_(p, IFGF_STAGE_LEAF_NODES, st, D);
            k_leaf_nodes<T, PS, PA, RB><<<grid_for((size_t)hp.L[D].nslots * P), kBlock, 0, st>>>(
                kc, p.L[D], p.pts, (const C*)p.dens_m, (C*)p.F[D], nullptr, 0);
        }
    hipError_t e;
    if (two && (e = hipEventRecord(ev_ready(p, D), st)) != hipSuccess) return e;
    for (int d = D; d >= 3; --d) {
        if (two && (e = hipStreamWaitEvent(sd, ev_ready(p, d), 0)) != hipSuccess) return e;
        cousin_stage<T, PS, PA, RB>(p, kc, d, grad, sd);
        if (two && (e = hipEventRecord(ev_read(p, d), sd)) != hipSuccess) return e;
        if (d > 3 && !reuse && hp.L[d - 1].nslots > 0)
            {
                // the nearest finer level whose buffer this step overwrites
                // (its cousin evaluation is the last reader on the side stream)
                if (two)
                    for (int dd = d + 1; dd <= D; ++dd)
                        if (p.F[dd] == p.F[d - 1]) {
                            if ((e = hipStreamWaitEvent(st, ev_read(p, dd), 0)) != hipSuccess) return e;
                            break;
                        }
                {
                    StageTimer tm_(p, IFGF_STAGE_CHILD_TO_PARENT, st, d);
                    c2p_launch<T, PS, PA, RB>(p, kc, d, c2p_variant<T, PS, PA, RB>(p, d), st);
                }
                // adaptive octree: the leaf boxes of level d - 1 have no
                // children; their cone values come from their own sources
                // (over the zeros the step above left in their slots)
                const LevelDev& Lq = p.L[d - 1];
                if (Lq.nleaf_slots > 0) {
                    StageTimer tm_(p, IFGF_STAGE_LEAF_NODES, st, d - 1);
                    k_leaf_nodes<T, PS, PA, RB><<<grid_for((size_t)Lq.nleaf_slots * P), kBlock, 0, st>>>(
                        kc, Lq, p.pts, (const C*)p.dens_m, (C*)p.F[d - 1], Lq.leaf_slots, Lq.nleaf_slots);
                }
            }
        if (two && d > 3 && (e = hipEventRecord(ev_ready(p, d - 1), st)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

template <typename T, int PS, int PA, int RB>
hipError_t apply_pass(DevicePlan& p, const void* dens, int nrhs, int r0, void* out, bool adj, hipStream_t st)
{
    const int n = (int)p.hp.n;
    using C = cpx<T>;
    // the adjoint conjugates every factor e^{i k .}: the phases use -k, and
    // the tabulated centred factors and ratios are conjugated (kc.adj)
    KernelConsts kc{make_cheb_nodes(p.hp.ps), make_cheb_nodes(p.hp.pang), adj ? -p.hp.kappa : p.hp.kappa, n, p.miss,
                    adj ? 1 : 0, p.hp.ps, p.hp.pang};
    hipError_t e;
    // (a capture records the side stream's work too: it joins the capture
    // through the first event wait and leaves it through the last; the side
    // stream and its events exist by then, made by run_prepare)
    const bool two = !p.no_alloc && side_stream_enabled() &&
                     (p.capturing ? p.side != nullptr : ensure_side(p) == hipSuccess);
    hipStream_t sd = two ? p.side : st;
    {
        StageTimer tm_(p, IFGF_STAGE_PERMUTE_IN, st);
        // forward: sources -> targets; adjoint: targets -> sources
        const Window w = adj ? target_window(p) : source_window(p);
        k_permute_in<T, RB><<<grid_for(n), kBlock, 0, st>>>((const C*)dens, (C*)p.dens_m, p.perm, n, w, nrhs, r0);
    }
    if (two) {
        if ((e = hipEventRecord(p.sync_ev[0], st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(sd, p.sync_ev[0], 0)) != hipSuccess) return e;
    }
    {
        StageTimer tm_(p, IFGF_STAGE_NEARFIELD, sd);
        k_nearfield<T, RB><<<grid_for(n), kBlock, 0, sd>>>(kc, p.L[p.hp.D], p.pts, (const C*)p.dens_m, (C*)p.out_m);
    }
    e = upward_and_eval<T, PS, PA, RB>(p, kc, st, false, false, sd);
    if (e != hipSuccess) return e;
    if (two) {
        if ((e = hipEventRecord(p.sync_ev[1], sd)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st, p.sync_ev[1], 0)) != hipSuccess) return e;
    }
    {
        StageTimer tm_(p, IFGF_STAGE_PERMUTE_OUT, st);
        const Window w = adj ? source_window(p) : target_window(p);
        k_permute_out<T, RB><<<grid_for((size_t)w.wn), kBlock, 0, st>>>((const C*)p.out_m, (C*)out, p.iperm, w, nrhs,
                                                                        r0);
    }
    return hipGetLastError();
}

template <typename T, int PS, int PA, int RB>
hipError_t grad_pass(DevicePlan& p, const void* dens, const void* gout, int nrhs, int r0, double* grad, bool reuse,
                     hipStream_t st)
{
    const int n = (int)p.hp.n;
    using C = cpx<T>;
    KernelConsts kc{make_cheb_nodes(p.hp.ps), make_cheb_nodes(p.hp.pang), p.hp.kappa, n, p.miss, 0, p.hp.ps,
                    p.hp.pang};
    if (!reuse)
        {
            StageTimer tm_(p, IFGF_STAGE_PERMUTE_IN, st);
            k_permute_in<T, RB><<<grid_for(n), kBlock, 0, st>>>((const C*)dens, (C*)p.dens_m, p.perm, n,
                                                                source_window(p), nrhs, r0);
        }
    {
        StageTimer tm_(p, IFGF_STAGE_PERMUTE_IN, st);
        k_permute_in<T, RB><<<grid_for(n), kBlock, 0, st>>>((const C*)gout, (C*)p.gout_m, p.perm, n,
                                                            target_window(p), nrhs, r0);
    }
    // the near-field and cousin gradients on the side stream, as in apply_pass
    hipError_t e;
    const bool two = !p.no_alloc && side_stream_enabled() &&
                     (p.capturing ? p.side != nullptr : ensure_side(p) == hipSuccess);
    hipStream_t sd = two ? p.side : st;
    if (two) {
        if ((e = hipEventRecord(p.sync_ev[0], st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(sd, p.sync_ev[0], 0)) != hipSuccess) return e;
    }
    {
        StageTimer tm_(p, IFGF_STAGE_NEAR_GRAD, sd);
        k_near_grad<T, RB><<<grid_for(n), kBlock, 0, sd>>>(kc, p.L[p.hp.D], p.pts, (const C*)p.dens_m,
                                                            (const C*)p.gout_m, p.grad_m);
    }
    e = upward_and_eval<T, PS, PA, RB>(p, kc, st, true, reuse, sd);
    if (e != hipSuccess) return e;
    if (two) {
        if ((e = hipEventRecord(p.sync_ev[1], sd)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st, p.sync_ev[1], 0)) != hipSuccess) return e;
    }
    {
        StageTimer tm_(p, IFGF_STAGE_PERMUTE_GRAD, st);
        const Window w = target_window(p);
        // passes after the first add their right-hand sides' share
        k_permute_grad<<<grid_for((size_t)w.wn), kBlock, 0, st>>>(p.grad_m, grad, p.iperm, w, r0 > 0 ? 1 : 0);
    }
    return hipGetLastError();
}

template <typename T, int PS, int PA>
hipError_t apply_t(DevicePlan& p, const void* dens, int nrhs, void* out, bool adj, hipStream_t st)
{
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPass) {
        int rb = rb_for(std::min(kMaxRhsPass, nrhs - r0));
        bool store = p.ws_store_pref && nrhs <= kMaxRhsPass;
        hipError_t e = ensure_workspace<T>(p, rb, store, nullptr);
        if (e != hipSuccess) return e;
        if (rb == 1) e = apply_pass<T, PS, PA, 1>(p, dens, nrhs, r0, out, adj, st);
        else if (rb == 4) e = apply_pass<T, PS, PA, 4>(p, dens, nrhs, r0, out, adj, st);
        else e = apply_pass<T, PS, PA, 16>(p, dens, nrhs, r0, out, adj, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------ the no-allocation apply

// Scratch of ifgf_apply_noalloc: the workspaces of an apply (densities and
// output in Morton order, two cone-value buffers, cousin-pair values) carved
// from one static device array.  Each GPU the library runs on holds its own
// copy until the process ends; every no-allocation call on a GPU shares it.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

// Address of this GPU's scratch array, taken once per device with that
// device current (host code never passes the array's name to a kernel: it is
// a host-side stand-in, not a device address).
static hipError_t scratch_address(int device, void** ptr)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void* q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = q;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

// Bytes of the no-allocation workspaces (256-byte aligned parts): densities
// and output [n][rb], two cone-value buffers [slots][P][rb], pair values.
static size_t noalloc_parts(const DevicePlan& p, int nrhs, size_t* b_dens, size_t* b_cone, size_t* b_pval)
{
    const HostPlan& hp = p.hp;
    const size_t rb = (size_t)rb_for(std::min(kMaxRhsPass, nrhs));
    const size_t ce = p.precision == IFGF_MIXED ? 8 : 16;
    size_t maxs = 0;
    for (int d = 3; d <= hp.D; ++d) maxs = std::max(maxs, (size_t)hp.L[d].nslots);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    *b_dens = up((size_t)hp.n * rb * ce);
    *b_cone = up(maxs * hp.P * rb * ce);
    *b_pval = up((size_t)p.max_pairs * rb * ce);
    return 2 * *b_dens + 2 * *b_cone + *b_pval;
}

template <typename T, int PS, int PA>
hipError_t apply_noalloc_t(DevicePlan& p, const void* dens, int nrhs, void* out, bool adj, hipStream_t st,
                           void* base)
{
    const HostPlan& hp = p.hp;
    size_t b_dens, b_cone, b_pval;
    if (noalloc_parts(p, nrhs, &b_dens, &b_cone, &b_pval) > kScratchBytes) return hipErrorOutOfMemory;
    // the plan's own workspaces are set aside (untouched) for the call
    void* s_dens = p.dens_m;
    void* s_out = p.out_m;
    void* s_pval = p.pval;
    const int64_t s_pval_pairs = p.pval_pairs;
    void* s_F[IFGF_MAX_LEVELS + 1];
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) s_F[d] = p.F[d];
    const bool s_prof = p.profiling;
    unsigned char* q = (unsigned char*)base;
    p.dens_m = q;
    p.out_m = q + b_dens;
    void* cone[2] = {q + 2 * b_dens, q + 2 * b_dens + b_cone};
    p.pval = p.max_pairs > 0 ? (void*)(q + 2 * b_dens + 2 * b_cone) : nullptr;
    p.pval_pairs = p.max_pairs;   // the scratch holds the tabulated levels' pairs only
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) p.F[d] = d >= 3 && d <= hp.D ? cone[d & 1] : nullptr;
    p.no_alloc = true;
    p.profiling = false;   // stage timers would create events
    hipError_t e = hipSuccess;
    for (int r0 = 0; r0 < nrhs && e == hipSuccess; r0 += kMaxRhsPass) {
        const int rbp = rb_for(std::min(kMaxRhsPass, nrhs - r0));
        if (rbp == 1) e = apply_pass<T, PS, PA, 1>(p, dens, nrhs, r0, out, adj, st);
        else if (rbp == 4) e = apply_pass<T, PS, PA, 4>(p, dens, nrhs, r0, out, adj, st);
        else e = apply_pass<T, PS, PA, 16>(p, dens, nrhs, r0, out, adj, st);
    }
    p.no_alloc = false;
    p.profiling = s_prof;
    p.dens_m = s_dens;
    p.out_m = s_out;
    p.pval = s_pval;
    p.pval_pairs = s_pval_pairs;
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) p.F[d] = s_F[d];
    return e;
}

template <typename T, int PS, int PA>
hipError_t grad_t(DevicePlan& p, const void* dens, const void* gout, int nrhs, double* grad, bool reuse,
                  hipStream_t st)
{
    // passes of at most 16 right-hand sides; the stored cone values can only
    // serve a single pass
    if (nrhs > kMaxRhsPass) reuse = false;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPass) {
        const int rb = rb_for(std::min(kMaxRhsPass, nrhs - r0));
        bool fresh = false;
        const bool store = p.ws_store_pref && nrhs <= kMaxRhsPass;
        hipError_t e = ensure_workspace<T>(p, rb, store, &fresh);
        if (e != hipSuccess) return e;
        if (fresh) reuse = false;
        if (rb == 1) e = grad_pass<T, PS, PA, 1>(p, dens, gout, nrhs, r0, grad, reuse, st);
        else if (rb == 4) e = grad_pass<T, PS, PA, 4>(p, dens, gout, nrhs, r0, grad, reuse, st);
        else e = grad_pass<T, PS, PA, 16>(p, dens, gout, nrhs, r0, grad, reuse, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int PS, int PA, int RB>
hipError_t autotune_t(DevicePlan& p, hipStream_t st)
{
    const HostPlan& hp = p.hp;
    const int D = hp.D;
    const int P = hp.P;
    using C = cpx<T>;
    hipError_t e = ensure_workspace<T>(p, RB, p.ws_store_pref, nullptr);
    if (e != hipSuccess) return e;
    p.stored_valid = false;
    if (D < 4) return hipSuccess;
    const bool prof = p.profiling;
    p.profiling = false;
    KernelConsts kc{make_cheb_nodes(hp.ps), make_cheb_nodes(hp.pang), hp.kappa, (int)hp.n, p.miss, 0, hp.ps,
                    hp.pang};
    if ((e = hipMemsetAsync(p.dens_m, 0, (size_t)hp.n * RB * sizeof(C), st)) != hipSuccess) return e;
    if (hp.L[D].nslots > 0)
        k_leaf_nodes<T, PS, PA, RB><<<grid_for((size_t)hp.L[D].nslots * P), kBlock, 0, st>>>(
            kc, p.L[D], p.pts, (const C*)p.dens_m, (C*)p.F[D], nullptr, 0);
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    for (int d = D; d >= 4 && e == hipSuccess; --d) {
        if (hp.L[d - 1].nslots == 0) continue;
        int v[kC2PVariants];
        const int nv = c2p_candidates<T, PS, PA, RB>(p, d, v);
        int best = c2p_default<T, PS, PA, RB>(p, d);
        float best_ms = 1e30f;
        for (int i = 0; i < nv && e == hipSuccess; ++i) {
            float ms = 1e30f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                (void)hipEventRecord(e0, st);
                c2p_launch<T, PS, PA, RB>(p, kc, d, v[i], st);
                (void)hipEventRecord(e1, st);
                if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
                if ((e = hipGetLastError()) != hipSuccess) break;
                float t = 0.f;
                (void)hipEventElapsedTime(&t, e0, e1);
                ms = t < ms ? t : ms;
            }
            if (autotune_verbose())
                std::fprintf(stderr, "autotune: level %d rb %d variant %d: %.3f ms\n", d, RB, v[i], (double)ms);
            if (ms < best_ms) {
                best_ms = ms;
                best = v[i];
            }
        }
        if (e != hipSuccess) break;
        p.c2p_choice[rb_index(RB)][d] = best;
        c2p_launch<T, PS, PA, RB>(p, kc, d, best, st);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p.profiling = prof;
    ++p.tune_gen;
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

template <typename T, int PS, int PA>
hipError_t autotune_rb(DevicePlan& p, int rb, hipStream_t st)
{
    if (rb == 1) return autotune_t<T, PS, PA, 1>(p, st);
    if (rb == 4) return autotune_t<T, PS, PA, 4>(p, st);
    return autotune_t<T, PS, PA, 16>(p, st);
}

template <typename T, int PS, int PA>
int candidates_t(const DevicePlan& p, int rb, int d, int* v)
{
    if (rb == 1) return c2p_candidates<T, PS, PA, 1>(p, d, v);
    if (rb == 4) return c2p_candidates<T, PS, PA, 4>(p, d, v);
    return c2p_candidates<T, PS, PA, 16>(p, d, v);
}

template <typename T, int PS, int PA>
int choice_t(const DevicePlan& p, int rb, int d)
{
    if (rb == 1) return c2p_variant<T, PS, PA, 1>(p, d);
    if (rb == 4) return c2p_variant<T, PS, PA, 4>(p, d);
    return c2p_variant<T, PS, PA, 16>(p, d);
}

}  // namespace

hipError_t run_prepare(DevicePlan& p, int nrhs)
{
    const int rb = rb_for(std::min(kMaxRhsPass, nrhs));
    const bool store = p.ws_store_pref && nrhs <= kMaxRhsPass;
    if (side_stream_enabled()) {
        hipError_t e = ensure_side(p);
        if (e != hipSuccess) return e;
    }
    return p.precision == IFGF_MIXED ? ensure_workspace<float>(p, rb, store, nullptr)
                                     : ensure_workspace<double>(p, rb, store, nullptr);
}

void note_apply(DevicePlan& p, const void* dens, int nrhs, bool adj)
{
    p.stored_valid = p.ws_store && !adj && nrhs <= kMaxRhsPass && p.ws_rb == rb_for(nrhs);
    p.stored_dens = dens;
    p.stored_nrhs = nrhs;
}

hipError_t run_autotune(DevicePlan& p, int nrhs, hipStream_t st)
{
    const int rb = rb_for(std::min(kMaxRhsPass, nrhs));
    const int ps = p.hp.ps, pa = p.hp.pang;
    const bool mixed = p.precision == IFGF_MIXED;
    if (ps == 3 && pa == 5) return mixed ? autotune_rb<float, 3, 5>(p, rb, st) : autotune_rb<double, 3, 5>(p, rb, st);
    if (ps == 4 && pa == 6) return mixed ? autotune_rb<float, 4, 6>(p, rb, st) : autotune_rb<double, 4, 6>(p, rb, st);
    if (ps == 2 && pa == 3) return mixed ? autotune_rb<float, 2, 3>(p, rb, st) : autotune_rb<double, 2, 3>(p, rb, st);
    if (any_degrees(ps, pa)) return mixed ? autotune_rb<float, 0, 0>(p, rb, st) : autotune_rb<double, 0, 0>(p, rb, st);
    return hipErrorInvalidValue;
}

int kernel_candidates(const DevicePlan& p, int nrhs, int d, int* v)
{
    if (d < 4 || d > p.hp.D || p.hp.L[d - 1].nslots == 0 || p.host_only) return 0;
    const int rb = rb_for(std::min(kMaxRhsPass, nrhs));
    const int ps = p.hp.ps, pa = p.hp.pang;
    const bool mixed = p.precision == IFGF_MIXED;
    if (ps == 3 && pa == 5) return mixed ? candidates_t<float, 3, 5>(p, rb, d, v) : candidates_t<double, 3, 5>(p, rb, d, v);
    if (ps == 4 && pa == 6) return mixed ? candidates_t<float, 4, 6>(p, rb, d, v) : candidates_t<double, 4, 6>(p, rb, d, v);
    if (ps == 2 && pa == 3) return mixed ? candidates_t<float, 2, 3>(p, rb, d, v) : candidates_t<double, 2, 3>(p, rb, d, v);
    if (any_degrees(ps, pa)) return mixed ? candidates_t<float, 0, 0>(p, rb, d, v) : candidates_t<double, 0, 0>(p, rb, d, v);
    return 0;
}

bool set_kernel_choice(DevicePlan& p, int nrhs, int d, int variant)
{
    const int rbi = rb_index(rb_for(std::min(kMaxRhsPass, nrhs)));
    if (variant < 0) {
        if (d >= 0 && d <= IFGF_MAX_LEVELS) p.c2p_choice[rbi][d] = -1;
        return true;
    }
    int v[kC2PVariants];
    const int n = kernel_candidates(p, nrhs, d, v);
    for (int i = 0; i < n; ++i)
        if (v[i] == variant) {
            p.c2p_choice[rbi][d] = variant;
            return true;
        }
    return false;
}

int kernel_choice(const DevicePlan& p, int nrhs, int d)
{
    if (d < 4 || d > p.hp.D || p.hp.L[d - 1].nslots == 0 || p.host_only) return -1;
    const int rb = rb_for(std::min(kMaxRhsPass, nrhs));
    const int ps = p.hp.ps, pa = p.hp.pang;
    const bool mixed = p.precision == IFGF_MIXED;
    if (ps == 3 && pa == 5) return mixed ? choice_t<float, 3, 5>(p, rb, d) : choice_t<double, 3, 5>(p, rb, d);
    if (ps == 4 && pa == 6) return mixed ? choice_t<float, 4, 6>(p, rb, d) : choice_t<double, 4, 6>(p, rb, d);
    if (ps == 2 && pa == 3) return mixed ? choice_t<float, 2, 3>(p, rb, d) : choice_t<double, 2, 3>(p, rb, d);
    if (any_degrees(ps, pa)) return mixed ? choice_t<float, 0, 0>(p, rb, d) : choice_t<double, 0, 0>(p, rb, d);
    return -1;
}

hipError_t run_apply(DevicePlan& p, const void* dens, int nrhs, void* out, bool adj, hipStream_t st)
{
    const int ps = p.hp.ps, pa = p.hp.pang;
    hipError_t e;
    bool mixed = p.precision == IFGF_MIXED;
    if (ps == 3 && pa == 5)
        e = mixed ? apply_t<float, 3, 5>(p, dens, nrhs, out, adj, st) : apply_t<double, 3, 5>(p, dens, nrhs, out, adj, st);
    else if (ps == 4 && pa == 6)
        e = mixed ? apply_t<float, 4, 6>(p, dens, nrhs, out, adj, st) : apply_t<double, 4, 6>(p, dens, nrhs, out, adj, st);
    else if (ps == 2 && pa == 3)
        e = mixed ? apply_t<float, 2, 3>(p, dens, nrhs, out, adj, st) : apply_t<double, 2, 3>(p, dens, nrhs, out, adj, st);
    else if (any_degrees(ps, pa))
        e = mixed ? apply_t<float, 0, 0>(p, dens, nrhs, out, adj, st) : apply_t<double, 0, 0>(p, dens, nrhs, out, adj, st);
    else
        return hipErrorInvalidValue;
    if (e == hipSuccess) note_apply(p, dens, nrhs, adj);
    return e;
}

hipError_t scratch_init(int device) {
    void* q = nullptr;
    return scratch_address(device, &q);
}

size_t scratch_bytes() { return kScratchBytes; }

size_t noalloc_bytes(const DevicePlan& p, int nrhs)
{
    size_t a, b, c;
    return noalloc_parts(p, nrhs, &a, &b, &c);
}

hipError_t run_apply_noalloc(DevicePlan& p, const void* dens, int nrhs, void* out, bool adj, hipStream_t st)
{
    void* base = nullptr;
    hipError_t e = scratch_address(p.device, &base);
    if (e != hipSuccess) return e;
    const int ps = p.hp.ps, pa = p.hp.pang;
    const bool mixed = p.precision == IFGF_MIXED;
    if (ps == 3 && pa == 5)
        return mixed ? apply_noalloc_t<float, 3, 5>(p, dens, nrhs, out, adj, st, base)
                     : apply_noalloc_t<double, 3, 5>(p, dens, nrhs, out, adj, st, base);
    if (ps == 4 && pa == 6)
        return mixed ? apply_noalloc_t<float, 4, 6>(p, dens, nrhs, out, adj, st, base)
                     : apply_noalloc_t<double, 4, 6>(p, dens, nrhs, out, adj, st, base);
    if (ps == 2 && pa == 3)
        return mixed ? apply_noalloc_t<float, 2, 3>(p, dens, nrhs, out, adj, st, base)
                     : apply_noalloc_t<double, 2, 3>(p, dens, nrhs, out, adj, st, base);
    if (any_degrees(ps, pa))
        return mixed ? apply_noalloc_t<float, 0, 0>(p, dens, nrhs, out, adj, st, base)
                     : apply_noalloc_t<double, 0, 0>(p, dens, nrhs, out, adj, st, base);
    return hipErrorInvalidValue;
}

hipError_t run_grad(DevicePlan& p, const void* dens, const void* gout, int nrhs, double* grad, bool reuse,
                    hipStream_t st)
{
    const int ps = p.hp.ps, pa = p.hp.pang;
    bool mixed = p.precision == IFGF_MIXED;
    reuse = reuse && nrhs <= kMaxRhsPass && p.ws_store && p.stored_valid && p.stored_dens == dens &&
            p.stored_nrhs == nrhs && p.ws_rb == rb_for(nrhs);
    hipError_t e;
    if (ps == 3 && pa == 5)
        e = mixed ? grad_t<float, 3, 5>(p, dens, gout, nrhs, grad, reuse, st) : grad_t<double, 3, 5>(p, dens, gout, nrhs, grad, reuse, st);
    else if (ps == 4 && pa == 6)
        e = mixed ? grad_t<float, 4, 6>(p, dens, gout, nrhs, grad, reuse, st) : grad_t<double, 4, 6>(p, dens, gout, nrhs, grad, reuse, st);
    else if (ps == 2 && pa == 3)
        e = mixed ? grad_t<float, 2, 3>(p, dens, gout, nrhs, grad, reuse, st) : grad_t<double, 2, 3>(p, dens, gout, nrhs, grad, reuse, st);
    else if (any_degrees(ps, pa))
        e = mixed ? grad_t<float, 0, 0>(p, dens, gout, nrhs, grad, reuse, st) : grad_t<double, 0, 0>(p, dens, gout, nrhs, grad, reuse, st);
    else
        return hipErrorInvalidValue;
    if (e == hipSuccess && p.ws_store && nrhs <= kMaxRhsPass) {
        // the stored cone values now hold these densities (reused or rebuilt)
        p.stored_valid = true;
        p.stored_dens = dens;
        p.stored_nrhs = nrhs;
    }
    return e;
}

}  // namespace ifgf
