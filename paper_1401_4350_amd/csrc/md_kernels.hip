// HIP kernels for gfx950: cell-list counting sort, Verlet-list build,
// vertex and edge pair-force decompositions, velocity-Verlet integration and
// deterministic energy reduction.
//
// Layout: particle records are packed 32-byte double4 (x, y, z, unused) in
// cell-sorted slot order, so one neighbour gather touches one 32-byte sector;
// the full Verlet list is tiled (list_row / list_off): for every tile of 64
// particles, rows of four entries per particle, so the lanes of a wavefront
// read consecutive words; the half list is CSR by row.  No kernel here uses
// matrix cores: the pair step is a gather plus a short scalar formula per
// pair, not a dense contraction.
//
// Every kernel body is a __device__ function of (system, logical block, block
// count); the single-system __global__ wrappers pass blockIdx (re-indexed per
// XCD where locality matters) and the batched wrappers (kb_*) pass the block
// that the batch's block map assigns.
#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "md_internal.h"

namespace md {

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------

// Workgroups are handed to the eight XCDs round-robin (block b runs on XCD
// b % 8).  Re-index so that every XCD walks a contiguous range of logical
// blocks: neighbouring particles (and their neighbour gathers) then share one
// XCD's L2 instead of being spread over all eight.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int nx = 8;
    int q = nb / nx, r = nb % nx;
    int x = b % nx, k = b / nx;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ double wrap_delta(double d, double box, double inv_box) {
    return d - box * rint(d * inv_box);
}

// Positions are kept unwrapped between list builds (they move by less than
// half a skin), and wrapped into [0, L) when the cells are rebuilt.  A list
// entry therefore fixes the periodic image of the pair for the lifetime of the
// list: entry = slot j | (s_x + 1) << 24 | (s_y + 1) << 26 | (s_z + 1) << 28,
// with the separation x_j - x_i + s L.  One select per axis replaces the
// divide-and-round of the minimum-image convention in the hot loops.
constexpr int kSlotBits = 24;
constexpr int kSlotMask = (1 << kSlotBits) - 1;

__device__ __forceinline__ int entry_slot(int e) { return e & kSlotMask; }

// Full lists are stored per tile: entry k of particle i (tile t = i / kTile,
// p = i % kTile) sits at word ((t * mcap + k / 4) * kTile + p) * 4 + k % 4.
// A tile's lists are one contiguous block, and four lanes that share a
// particle read 16 consecutive bytes, so a wavefront's load is one contiguous
// 256-byte run.  list_row(s, i) points at entry 0 of particle i; entry k is
// at offset list_off(k).
__device__ __forceinline__ const int* list_row(const Sys& s, int i) {
    return s.nbr + (((size_t)(i / kTile) * s.mcap) * kTile + (i % kTile)) * 4;
}
__device__ __forceinline__ int* list_row_w(const Sys& s, int i) {
    return s.nbr + (((size_t)(i / kTile) * s.mcap) * kTile + (i % kTile)) * 4;
}
__device__ __forceinline__ size_t list_off(int k) { return (size_t)(k >> 2) * (kTile * 4) + (k & 3); }
// A staged tile's entries are 16-bit indices into its region (the region
// copy carries the periodic image), eight per 16-byte row: entry k of
// particle i at 16-bit word ((t * mcap + k / 8) * kTile + p) * 8 + k % 8 of
// the same block, so the tile uses ceil(cap / 8) of its rows and a lane's
// 32-bit load brings two entries.
__device__ __forceinline__ const uint16_t* list_row16(const Sys& s, int i) {
    return reinterpret_cast<const uint16_t*>(list_row(s, i));
}
__device__ __forceinline__ size_t list_off16(int k) { return (size_t)(k >> 3) * (kTile * 8) + (k & 7); }
// Edge index of full-list entry k of particle i (deterministic edge mode):
// word list_off(k) of eidx_row(s, i), laid out like 32-bit list entries.
__device__ __forceinline__ int* eidx_row(const Sys& s, int i) {
    return s.eidx + (((size_t)(i / kTile) * s.mcap) * kTile + (i % kTile)) * 4;
}

__device__ __forceinline__ double image(int e, int axis, double box) {
    int c = (e >> (kSlotBits + 2 * axis)) & 3;
    return c == 1 ? 0.0 : (c == 0 ? -box : box);
}

__device__ __forceinline__ int image_code(double d, double inv_box) {
    return (int)(-rint(d * inv_box)) + 1;
}

__device__ __forceinline__ double wrap_box(double y, double L) {
    if (y >= L) y -= L;
    if (y < 0) y += L;
    return y;
}

// 1 / a from the hardware reciprocal (relative error 4.6e-8 on gfx950) and
// one Newton step: relative error below 2.2e-15 over the r^2 range of the
// pair maths (measured against a long-double reference on 4M arguments).
__device__ __forceinline__ double rcp_nr(double a) {
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ float rcp_nr(float a) {
    float y = __builtin_amdgcn_rcpf(a);
    float e = fmaf(-a, y, 1.0f);
    return fmaf(y, e, y);
}

__device__ __forceinline__ int cell_coord(double x, double cell_inv, int nc) {
    int c = (int)(x * cell_inv);
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}


// ---------------------------------------------------------------------------
// Pair potentials (arithmetic type R; accumulation is the caller's)
// ---------------------------------------------------------------------------

// Truncated-and-shifted Lennard-Jones (Eq. 1).  Returns F/r such that the
// force on j is (F/r) * (x_j - x_i); *v gets V(r) - V(r_c).
template <typename R>
__device__ __forceinline__ R lj_fr(R r2, const LJc<R>& c, R* v) {
    R inv = R(1) / r2;
    R s2 = c.sig2 * inv;
    R s6 = s2 * s2 * s2;
    if (v) *v = c.eps4 * (s6 * s6 - s6) - c.vshift;
    return c.eps24 * (R(2) * s6 * s6 - s6) * inv;
}

template <typename R>
struct V3 {
    R x, y, z;
};
template <typename R>
__device__ __forceinline__ R dot3(const V3<R>& a, const V3<R>& b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}

// The patch directions of a particle with orientation q = (w, x, y, z).
// Model 0: the four tetrahedral directions u_a = R(q) e_a with
// e_a = (+-1, +-1, +-1)/sqrt(3) having an even number of minus signs, i.e. sums
// and differences of R's columns.  Model 1: the two poles +-R(q) e_z (u[2],
// u[3] unused).
template <typename R>
__device__ __forceinline__ void patch_dirs(const double4& q, V3<R> u[4], int model = 0) {
    R w = (R)q.x, x = (R)q.y, y = (R)q.z, z = (R)q.w;
    V3<R> c0 = {R(1) - R(2) * (y * y + z * z), R(2) * (x * y + w * z), R(2) * (x * z - w * y)};
    V3<R> c1 = {R(2) * (x * y - w * z), R(1) - R(2) * (x * x + z * z), R(2) * (y * z + w * x)};
    V3<R> c2 = {R(2) * (x * z + w * y), R(2) * (y * z - w * x), R(1) - R(2) * (x * x + y * y)};
    if (model == 1) {
        u[0] = c2;
        u[1] = {-c2.x, -c2.y, -c2.z};
        u[2] = u[3] = {R(0), R(0), R(0)};
        return;
    }
    const R k = R(0.57735026918962576451);  // 1/sqrt(3)
    u[0] = {k * (c0.x + c1.x + c2.x), k * (c0.y + c1.y + c2.y), k * (c0.z + c1.z + c2.z)};
    u[1] = {k * (c0.x - c1.x - c2.x), k * (c0.y - c1.y - c2.y), k * (c0.z - c1.z - c2.z)};
    u[2] = {k * (-c0.x + c1.x - c2.x), k * (-c0.y + c1.y - c2.y), k * (-c0.z + c1.z - c2.z)};
    u[3] = {k * (-c0.x - c1.x + c2.x), k * (-c0.y - c1.y + c2.y), k * (-c0.z - c1.z + c2.z)};
}

__device__ __forceinline__ float exp_r(float a) { return __expf(a); }
__device__ __forceinline__ double exp_r(double a) { return exp(a); }

// Two-patch pair (the model of Eqs. 2-4 with M = 2 polar patches): the core
// (sigma/r)^200 plus, for each of the four patch pairs (a, b) with
// s = |d + delta (u_j^b - u_i^a)| below rpc, -eps_p exp(-(s/w)^10 / 2).
// d, r2, outputs and torques as for patchy_pair below.  The core (steep: its
// force changes by 200 ulp per ulp of r^2) and the geometry are FP64 in every
// precision; R is the type of the scalar factor of each patch term.
template <typename R>
__device__ __forceinline__ void patchy2_pair(const V3<double>& d, double r2, const V3<double> ui[4],
                                             const V3<double> uj[4], const Sys& s, V3<double>& fj,
                                             V3<double>& ti, V3<double>& tj, double& v) {
    const PatchyC<double>& c = s.p64;
    {   // (sigma^2/r^2)^100 by squaring; F_j = -dV/dr = 200 V_core d / r^2
        const double inv = 1.0 / r2;
        const double t = c.sig2 * inv;
        const double t2 = t * t, t4 = t2 * t2, t8 = t4 * t4, t16 = t8 * t8, t32 = t16 * t16;
        const double vc = (t32 * t32) * (t32 * t4);
        v += vc;
        const double fr = 200.0 * vc * inv;
        fj.x += fr * d.x;
        fj.y += fr * d.y;
        fj.z += fr * d.z;
    }
    const R inv_w2 = (R)c.inv_w2, eps_p = (R)c.eps_p;
#pragma unroll
    for (int a = 0; a < 2; a++) {
#pragma unroll
        for (int b = 0; b < 2; b++) {
            V3<double> dd64 = {d.x + c.delta * (uj[b].x - ui[a].x),
                               d.y + c.delta * (uj[b].y - ui[a].y),
                               d.z + c.delta * (uj[b].z - ui[a].z)};
            double s2 = dot3(dd64, dd64);
            if (c.rpc2 > 0.0 && !(s2 < c.rpc2)) continue;
            // the exponent reaches (0.18 / 0.12)^10 / 2 = 29 at the patch range,
            // so it is formed in FP64: its rounding error is the relative
            // error of the term
            const double x = s2 * c.inv_w2;  // (s/w)^2
            const double x4d = (x * x) * (x * x);
            const R x4 = (R)x4d;
            const R E = exp_r((R)(-0.5 * x4d * x));
            v -= (double)(eps_p * E);
            // dV/dd_ab = kk d_ab; -dV/du_i^a = delta kk d_ab = dV/du_j^b.  Only
            // the scalars are in R: the directions stay FP64, so the rounding
            // of a bonded pair's torque is relative to the torque itself.
            const double kk = (double)(R(5) * eps_p * E * x4 * inv_w2);
            const double m = c.delta * kk;
            fj.x -= kk * dd64.x;
            fj.y -= kk * dd64.y;
            fj.z -= kk * dd64.z;
            ti.x += m * (ui[a].y * dd64.z - ui[a].z * dd64.y);
            ti.y += m * (ui[a].z * dd64.x - ui[a].x * dd64.z);
            ti.z += m * (ui[a].x * dd64.y - ui[a].y * dd64.x);
            tj.x -= m * (uj[b].y * dd64.z - uj[b].z * dd64.y);
            tj.y -= m * (uj[b].z * dd64.x - uj[b].x * dd64.z);
            tj.z -= m * (uj[b].x * dd64.y - uj[b].y * dd64.x);
        }
    }
}

// Patchy pair: WCA core + sum over facing patch pairs of
// -eps_p exp(-|d_ab|^2 / w^2) * A(c_i^a) * A(c_j^b), A(c) = c^2 for c > 0.
// d = x_j - x_i (minimum image), r2 = |d|^2 < r_cut^2.  Outputs the force on j
// (fj, the force on i is -fj), the torques on i and j, and the pair energy.
// Torques come from the patch-vector gradients: tau = sum_a u_a x (-dV/du_a).
// The geometry (separation, patch directions, patch-patch offsets d_ab) and
// the WCA core are FP64 in every precision; R is the type of the Gaussian,
// the angular products and the gradient assembly of each patch pair.  (The
// force of a bonded pair is sensitive to its geometry: rounding the patch
// directions or the WCA factor near its zero to FP32 would cost more than the
// FP32 force budget.)
template <typename R>
__device__ __forceinline__ void patchy_pair(const V3<double>& d, double r2, const V3<double> ui[4],
                                            const V3<double> uj[4], const Sys& s, V3<double>& fj,
                                            V3<double>& ti, V3<double>& tj, double& v) {
    const PatchyC<double>& c = s.p64;
    fj = {0, 0, 0};
    ti = {0, 0, 0};
    tj = {0, 0, 0};
    v = 0;
    if (c.model == 1) {
        patchy2_pair<R>(d, r2, ui, uj, s, fj, ti, tj, v);
        return;
    }
    if (r2 < c.wca2) {
        double inv = 1.0 / r2;
        double s2 = c.sig2 * inv;
        double s6 = s2 * s2 * s2;
        v += c.eps4 * (s6 * s6 - s6) + c.eps;
        double fr = c.eps24 * (2.0 * s6 * s6 - s6) * inv;
        fj.x += fr * d.x;
        fj.y += fr * d.y;
        fj.z += fr * d.z;
    }
    double rinv = 1.0 / sqrt(r2);
    V3<double> h = {d.x * rinv, d.y * rinv, d.z * rinv};
    double ci[4], cj[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        ci[a] = dot3(ui[a], h);
        cj[a] = -dot3(uj[a], h);
    }
    const R delta = (R)c.delta, inv_w2 = (R)c.inv_w2, eps_p = (R)c.eps_p;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        if (!(ci[a] > 0.0)) continue;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            if (!(cj[b] > 0.0)) continue;
            V3<double> dd64 = {d.x + c.delta * (uj[b].x - ui[a].x),
                               d.y + c.delta * (uj[b].y - ui[a].y),
                               d.z + c.delta * (uj[b].z - ui[a].z)};
            double s2 = dot3(dd64, dd64);
            if (c.rpc2 > 0.0 && !(s2 < c.rpc2)) continue;
            // assembly in R from the FP64 geometry
            const R cia = (R)ci[a], cjb = (R)cj[b], rinvR = (R)rinv, r = (R)(r2 * rinv);
            const V3<R> dd = {(R)dd64.x, (R)dd64.y, (R)dd64.z};
            const V3<R> hh = {(R)h.x, (R)h.y, (R)h.z};
            const V3<R> ua = {(R)ui[a].x, (R)ui[a].y, (R)ui[a].z};
            const V3<R> ub = {(R)uj[b].x, (R)uj[b].y, (R)uj[b].z};
            R Ai = cia * cia, Aj = cjb * cjb;
            R g = -eps_p * exp_r((R)(-s2 * c.inv_w2));
            R G = g * Ai * Aj;
            v += (double)G;
            // gradient pieces: Gaussian (along d_ab) and the two cosines
            R kd = R(2) * G * inv_w2;           // Gaussian: dV/dr gets -kd d_ab
            R ki = g * Aj * R(2) * cia * rinvR;  // through c_i
            R kj = g * Ai * R(2) * cjb * rinvR;  // through c_j
            // dV/dr = -kd d_ab + ki (u_i - c_i h) + kj (-u_j - c_j h); F_j = -dV/dr
            fj.x += (double)(kd * dd.x - ki * (ua.x - cia * hh.x) + kj * (ub.x + cjb * hh.x));
            fj.y += (double)(kd * dd.y - ki * (ua.y - cia * hh.y) + kj * (ub.y + cjb * hh.y));
            fj.z += (double)(kd * dd.z - ki * (ua.z - cia * hh.z) + kj * (ub.z + cjb * hh.z));
            // -dV/du_i = -(delta kd d_ab + ki r h),  -dV/du_j = delta kd d_ab + kj r h
            V3<R> mi = {-(delta * kd * dd.x + ki * r * hh.x), -(delta * kd * dd.y + ki * r * hh.y),
                        -(delta * kd * dd.z + ki * r * hh.z)};
            V3<R> mj = {delta * kd * dd.x + kj * r * hh.x, delta * kd * dd.y + kj * r * hh.y,
                        delta * kd * dd.z + kj * r * hh.z};
            // torques: u x m with the FP64 direction (m nearly parallel to u for
            // a bonded patch, so the cross product cancels)
            const double mix = mi.x, miy = mi.y, miz = mi.z;
            const double mjx = mj.x, mjy = mj.y, mjz = mj.z;
            ti.x += ui[a].y * miz - ui[a].z * miy;
            ti.y += ui[a].z * mix - ui[a].x * miz;
            ti.z += ui[a].x * miy - ui[a].y * mix;
            tj.x += uj[b].y * mjz - uj[b].z * mjy;
            tj.y += uj[b].z * mjx - uj[b].x * mjz;
            tj.z += uj[b].x * mjy - uj[b].y * mjx;
        }
    }
}


// ---------------------------------------------------------------------------
// Control
// ---------------------------------------------------------------------------

__global__ void k_set_rebuild(Ctrl* c) { c->rebuild = 1; }

__global__ void k_clear_ctrl(Ctrl* c, int* sync) {
    for (int k = threadIdx.x; k < kSyncUses * kSyncInts; k += blockDim.x) sync[k] = 0;
    if (threadIdx.x != 0) return;
    c->rebuild = 0;
    c->overflow = 0;
    c->nonfinite = 0;
    c->max_count = 0;
    c->staged = 0;
    c->npairs = 0;
    c->rebuilds = 0;
    c->half_stale = 0;
    c->eidx_stale = 0;
    c->nonzero = 0;
    c->req[0] = c->req[1] = 0;  // launch ids start at 2
}

// True in the one workgroup, of the nb that call this with the same counter,
// that arrives last; that workgroup then sees the device-scope atomics and
// agent-scope stores every other one made before arriving.  Resets the
// counter for its next use.  Every thread of the workgroup must call it.
// True in the workgroup that finishes last of nb (workgroup bid of 0 .. nb-1).
// Two-level count over the counters `cnt` (kSyncInts ints, zero before and
// after).  It orders nothing beyond the count: a per-workgroup cache
// writeback (a device-scope release) costs about 20 ns per workgroup,
// serialised, so data the last workgroup reads from the others travels only
// through device-coherent accesses: atomic read-modify-writes, or
// device-scope atomic stores, which are complete once the barrier below has
// waited for the workgroup's memory operations, read back with device-scope
// atomic loads (coh_load).  Plain stores are seen by later kernels only.
__device__ __forceinline__ bool last_block(int* cnt, int bid, int nb) {
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int g = bid % kSyncFan;
        const int members = (nb - 1 - g) / kSyncFan + 1;  // workgroups of group g
        int last = 0;
        if (atomicAdd(&cnt[g * kSyncStride], 1) == members - 1) {
            atomicExch(&cnt[g * kSyncStride], 0);
            const int groups = nb < kSyncFan ? nb : kSyncFan;
            if (atomicAdd(&cnt[kSyncFan * kSyncStride], 1) == groups - 1) {
                atomicExch(&cnt[kSyncFan * kSyncStride], 0);
                last = 1;
            }
        }
        is_last = last;
    }
    __syncthreads();
    return is_last;
}

// Device-coherent store and load of an int (for last_block's epilogues).
__device__ __forceinline__ void coh_store(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int coh_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Cell-list counting sort.  Every kernel returns at once unless a rebuild is
// due, so the sequence can sit in every step without a host round trip.
// ---------------------------------------------------------------------------

// Exclusive prefix sum of a[0, len) by one workgroup, a[k] = load(k):
// emit(k, sum of a[0, k), a[k]) for every k, in chunks of kBlock * V
// elements (each thread V consecutive ones, all loads issued first).
// Returns the total.
template <int V, typename Load, typename Emit>
__device__ __forceinline__ long long block_scan(int len, Load load, Emit emit) {
    __shared__ long long sh[kBlock];
    const int t = threadIdx.x;
    long long base = 0;
    for (int c0 = 0; c0 < len; c0 += kBlock * V) {
        const int k0 = c0 + t * V;
        int v[V];
        if (k0 + V <= len) {  // whole run in range: every load issued before any wait
#pragma unroll
            for (int u = 0; u < V; u++) v[u] = load(k0 + u);
        } else {
#pragma unroll
            for (int u = 0; u < V; u++) v[u] = k0 + u < len ? load(k0 + u) : 0;
        }
        long long sum = 0;
#pragma unroll
        for (int u = 0; u < V; u++) sum += v[u];
        sh[t] = sum;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            long long w = t >= off ? sh[t - off] : 0;
            __syncthreads();
            sh[t] += w;
            __syncthreads();
        }
        long long run = base + sh[t] - sum;
#pragma unroll
        for (int u = 0; u < V; u++) {
            if (k0 + u < len) emit(k0 + u, run, v[u]);
            run += v[u];
        }
        base += sh[kBlock - 1];
        __syncthreads();  // sh is rewritten by the next chunk
    }
    return base;
}

// Exclusive scan of the cell counts into cell_start by one workgroup (the
// scatter pass clears the counts for the next build).  Sparse systems have
// several cells per particle, so the counts are read and the starts written
// coalesced (element c0 + u * kBlock + t by thread t), through an LDS tile in
// which each thread scans kCellRun consecutive counts.  The counts come from
// other workgroups' atomics: device-coherent loads.
constexpr int kCellRun = 16;
__device__ __forceinline__ int cell_lds(int p) { return p + p / 32; }  // pad: no bank conflicts

__device__ __forceinline__ void scan_cells(const Sys& s) {
    __shared__ int tile[kBlock * kCellRun + kBlock * kCellRun / 32];
    __shared__ long long part[kBlock];
    const int t = threadIdx.x, len = s.ncell;
    constexpr int C = kBlock * kCellRun;
    long long base = 0;
    for (int c0 = 0; c0 < len; c0 += C) {
        int v[kCellRun];
        if (c0 + C <= len) {
#pragma unroll
            for (int u = 0; u < kCellRun; u++) v[u] = coh_load(&s.ccount[c0 + u * kBlock + t]);
        } else {
#pragma unroll
            for (int u = 0; u < kCellRun; u++) {
                const int k = c0 + u * kBlock + t;
                v[u] = k < len ? coh_load(&s.ccount[k]) : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kCellRun; u++) tile[cell_lds(u * kBlock + t)] = v[u];
        __syncthreads();
        // thread t: counts t * kCellRun .. + kCellRun - 1 of the chunk
        int run[kCellRun];
        long long sum = 0;
#pragma unroll
        for (int u = 0; u < kCellRun; u++) {
            run[u] = tile[cell_lds(t * kCellRun + u)];
            sum += run[u];
        }
        part[t] = sum;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            long long w = t >= off ? part[t - off] : 0;
            __syncthreads();
            part[t] += w;
            __syncthreads();
        }
        long long r = base + part[t] - sum;
#pragma unroll
        for (int u = 0; u < kCellRun; u++) {
            const int c = run[u];
            tile[cell_lds(t * kCellRun + u)] = (int)r;
            r += c;
        }
        base += part[kBlock - 1];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kCellRun; u++) {
            const int k = c0 + u * kBlock + t;
            if (k < len) s.cstart[k] = tile[cell_lds(u * kBlock + t)];
        }
        __syncthreads();  // the tile and part are rewritten by the next chunk
    }
    if (t == 0) s.cstart[len] = (int)base;
}

// Bins every particle into its cell (counts by atomics; the atomic's return
// value is the particle's provisional rank in the cell); the workgroup that
// finishes last scans the counts into cell starts.  Lanes of a wavefront in
// the same cell share one atomic (particles arrive in slot order, so a
// wavefront holds few cells): one add of their number, then ranks by lane
// order.
__device__ __forceinline__ void b_cell_bin(const Sys& s, int bid, int nb) {
    if (!s.ctrl->rebuild) return;
    const int p = bid * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    int c = -1;
    if (p < s.n) {
        const double4 x = s.pos[p];
        const int cx = cell_coord(wrap_box(x.x, s.box), s.cell_inv, s.nc);
        const int cy = cell_coord(wrap_box(x.y, s.box), s.cell_inv, s.nc);
        const int cz = cell_coord(wrap_box(x.z, s.box), s.cell_inv, s.nc);
        c = (cz * s.nc + cy) * s.nc + cx;
        if (s.cell_rank) c = s.cell_rank[c];  // cells along a space-filling curve
        s.cell[p] = c;
    }
    // group the lanes by cell (no memory traffic), then one atomic per group,
    // all groups at once
    const unsigned long long below = (1ull << lane) - 1;
    unsigned long long todo = __ballot(c >= 0);
    int lead = lane, idx = 0, size = 0;
    while (todo) {
        const int l = __builtin_ctzll(todo);
        const int cl = __builtin_amdgcn_readlane(c, l);
        const unsigned long long same = __ballot(c == cl);
        if (c == cl) lead = l, idx = __builtin_popcountll(same & below);
        if (lane == l) size = __builtin_popcountll(same);
        todo &= ~same;
    }
    int base = 0;
    if (size > 0) base = atomicAdd(&s.ccount[c], size);
    base = __shfl(base, lead);
    if (p < s.n) s.rank[p] = base + idx;
    if (last_block(s.sync + kSyncBin * kSyncInts, bid, nb)) scan_cells(s);
}

__global__ __launch_bounds__(kBlock) void k_cell_bin(Sys s) { b_cell_bin(s, blockIdx.x, gridDim.x); }

__device__ __forceinline__ void b_cell_scatter(const Sys& s, int bid, int nb) {
    if (!s.ctrl->rebuild) return;
    int p = bid * kBlock + threadIdx.x;
    // the scan has read the counts: clear them for the next build
    for (int c = p; c < s.ncell; c += nb * kBlock) s.ccount[c] = 0;
    if (p >= s.n) return;
    s.order[s.cstart[s.cell[p]] + s.rank[p]] = p;
}

__global__ __launch_bounds__(kBlock) void k_cell_scatter(Sys s) {
    b_cell_scatter(s, blockIdx.x, gridDim.x);
}

// One lane per particle puts the members of every cell (scattered in atomic
// order) in ascending order of their previous slot, so the slot order, and
// every sum over a list, does not depend on atomic timing: particle p's rank
// is the number of members of its cell with a smaller previous slot.  Its
// records (position wrapped into the box, with its FP32 copy, velocity, id,
// orientation) are copied to the reorder buffers at its new slot.
__device__ __forceinline__ void b_cell_sort(const Sys& s, int bid) {
    const int p = bid * kBlock + threadIdx.x;
    if (p >= s.n) return;
    const int c = s.cell[p];
    const int b = s.cstart[c], m = s.cstart[c + 1] - b;
    int rank = 0;
    for (int k = 0; k < m; k += 4) {  // four members per round, loads first
        const int o0 = s.order[b + k];
        const int o1 = s.order[b + min(k + 1, m - 1)];
        const int o2 = s.order[b + min(k + 2, m - 1)];
        const int o3 = s.order[b + min(k + 3, m - 1)];
        rank += (o0 < p) + (k + 1 < m && o1 < p) + (k + 2 < m && o2 < p) + (k + 3 < m && o3 < p);
    }
    const int q = b + rank;
    const double4 x = s.pos[p];
    const double wx = wrap_box(x.x, s.box), wy = wrap_box(x.y, s.box), wz = wrap_box(x.z, s.box);
    s.tpos[q] = make_double4(wx, wy, wz, 0.0);
    s.tposf[q] = make_float4((float)wx, (float)wy, (float)wz, 0.f);
    s.tvel[q] = s.vel[p];
    s.tid[q] = s.id[p];
    if (s.pot == 1) {
        s.tquat[q] = s.quat[p];
        s.tangm[q] = s.angm[p];
    }
}

// ---------------------------------------------------------------------------
// Tile regions (one wavefront per tile of kTile consecutive slots).  The tile's
// home cells are a run of cell ids over at most two rows of cells; the 27-cell
// neighbourhood of a row run is, for each of the 9 surrounding rows, an
// x-interval of cells, i.e. a contiguous slot range, split in two where it
// crosses the periodic boundary.  Each range is recorded with the periodic
// image that places it next to the home cells, so the LDS copy can carry the
// image.  Tiles over more rows, or spanning a whole row, use global gathers.
// ---------------------------------------------------------------------------


// Wavefront prefix sum (exclusive) of v over the 64 lanes.
__device__ __forceinline__ int wave_excl_scan(int v, int lane) {
    int x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x - v;
}

// Region of one tile, computed by one wavefront.  Segment slots are fixed:
// two per (home row h, dz, dy), slot ((h * 3 + dz + 1) * 3 + dy + 1) * 2 + k,
// the second one empty unless the x-interval wraps the box, so the list
// build finds a cell's segment by index.  Lane q < 36 fills slot q; LDS bases
// and the copy chunks (runs of at most 64 slots) follow from wavefront prefix
// sums.  Runs after the scatter: the cell of new slot a is cell[order[a]].
__device__ __forceinline__ void b_tile_region(const Sys& s, int t) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nc = s.nc;
    if (nc < 3 || s.cell_order != 0) {  // gathers from global memory
        if (lane == 0) s.tile_nseg[t] = -1;
        return;
    }
    const int a = t * kTile;
    const int b = min(a + kTile, s.n) - 1;
    const int c0 = s.cell[s.order[a]], c1 = s.cell[s.order[b]];
    const int r0 = c0 / nc, r1 = c1 / nc;
    bool ok = r1 - r0 <= 1;
    const int nseg = r1 > r0 ? 36 : 18;
    int b0 = 0, b1 = 0, code = -1;  // this lane's segment: slots [b0, b1), image code
    bool bad = false;
    if (ok && lane < nseg) {
        const int h = lane / 18, dz = (lane / 6) % 3 - 1, dy = (lane / 2) % 3 - 1, k2 = lane & 1;
        const int r = r0 + h;
        const int xa = r == r0 ? c0 % nc : 0;
        const int xb = r == r1 ? c1 % nc : nc - 1;
        bad = xb - xa + 3 > nc;  // one row would need two x images
        const int y = r % nc, z = r / nc;
        auto wrapc = [&](int v) { return v < 0 ? 0 : (v >= nc ? 2 : 1); };  // shift -L, 0, +L
        const int rr = ((z + dz + nc) % nc) * nc + (y + dy + nc) % nc;
        const int yz = wrapc(y + dy) << 2 | wrapc(z + dz) << 4;
        const int lo = xa - 1, hi = xb + 1;
        int xl = 0, xh = -1;  // cell run [xl, xh] of this slot, empty if xh < xl
        if (lo < 0) {
            if (k2 == 0) xl = lo + nc, xh = nc - 1, code = yz | 0;
            else xl = 0, xh = hi, code = yz | 1;
        } else if (hi >= nc) {
            if (k2 == 0) xl = lo, xh = nc - 1, code = yz | 1;
            else xl = 0, xh = hi - nc, code = yz | 2;
        } else if (k2 == 0) {
            xl = lo, xh = hi, code = yz | 1;
        }
        if (!bad && xh >= xl) {
            b0 = s.cstart[rr * nc + xl];
            b1 = s.cstart[rr * nc + xh + 1];
        }
    }
    ok = ok && !__any(bad);
    const int len = b1 - b0;
    const int base = wave_excl_scan(len, lane);
    const int total = __shfl(base + len, kWave - 1);
    const int nch = (len + kWave - 1) / kWave;
    const int cbase = wave_excl_scan(nch, lane);
    const int nchk = __shfl(cbase + nch, kWave - 1);
    ok = ok && total <= s.lds_cap && nchk <= kChunkMax;
    if (!ok) {
        if (lane == 0) s.tile_nseg[t] = -1;
        return;
    }
    static_assert(kSegMax >= 36, "two home rows x 9 neighbour rows x 2 slots");
    if (lane < nseg) s.tile_seg[(size_t)t * kSegMax + lane] = make_int4(b0, b1, base, code);
    int4* chk = s.tile_chunk + (size_t)t * kChunkMax + cbase;
    for (int u = 0; u < nch; u++)
        chk[u] = make_int4(b0 + u * kWave, min(b1, b0 + (u + 1) * kWave), base + u * kWave, code);
    if (lane == 0) {
        s.tile_nchunk[t] = nchk;
        s.tile_row0[t] = r0;
        s.tile_nseg[t] = nseg;
    }
}

// Cell sort (the first sort_blocks workgroups, wavefronts striding over the
// cells) and tile regions (the rest, one wavefront per tile).
__device__ __forceinline__ void b_sort_tiles(const Sys& s, int bid, int nb) {
    if (!s.ctrl->rebuild) return;
    const int ns = sort_blocks(s);
    if (bid < ns) {
        b_cell_sort(s, bid);
    } else {
        const int t = (bid - ns) * (kBlock / kWave) + threadIdx.x / kWave;
        if (t < s.ntiles) b_tile_region(s, t);
    }
}

__global__ __launch_bounds__(kBlock) void k_sort_tiles(Sys s) { b_sort_tiles(s, blockIdx.x, gridDim.x); }


// Position of slot range [cb, ...) seen through image `code` inside a tile's
// LDS image: base + (cb - begin) of the segment that holds it, or -1.
__device__ __forceinline__ int tile_lds_base(const int4* seg, int nseg, int cb, int code) {
    for (int q = 0; q < nseg; q++) {
        int4 g = seg[q];
        if (g.w == code && cb >= g.x && cb < g.y) return g.z + (cb - g.x);
    }
    return -1;
}

// Packed half-list word of the patchy edge pass: partner not in the region.
constexpr int kNoRegion = 0xffff;
// The patchy edge pass goes by tiles (k_edge_patchy_tile) for the four-patch
// model from 256 tiles (16 384 particles) on; otherwise by 64-entry chunks
// (k_edge).  The two-patch chains give about one bonded partner per particle,
// so partners are hardly ever shared inside a tile and the tile's set-up and
// flush cost more than the global atomics they save (the tile pass measured
// 19 % slower there); small systems leave most of the chip idle, where the
// tile's serial set-up and flush show (33 against 25 us at 4 096 particles),
// while from 16 384 particles on the tile pass is 2-21 % faster.
constexpr int kPatchyTileMin = 256;
__device__ __host__ __forceinline__ bool patchy_edge_by_tile(const Sys& s) {
    return s.p64.model == 0 && s.ntiles >= kPatchyTileMin;
}
// Image code (two bits per axis, shift + 1) of a slot seen without a shift.
constexpr int kCodeHome = 1 | 1 << 2 | 1 << 4;

// ---------------------------------------------------------------------------
// Copy of a staged tile's region into LDS (list build and vertex pass).
// Wave v takes chunks v, v + 4, ... (runs of at most 64 slots with one image
// each) in batches of R; chunk descriptors are wave-uniform.  The loads of a
// batch are issued by region_issue and consumed by region_store, so a caller
// can put other loads in between: loads retire in order, so the first batch
// is issued before slower loads and stored right after them.
// LDS layout: one packed 24-byte record (x, y, z) per region slot, so a
// neighbour is one address and two reads (16 + 8 bytes), and the region of a
// typical tile leaves room for four workgroups per CU; slot `cap` is a
// padding particle far outside the box.
// ---------------------------------------------------------------------------

constexpr double kFar = 1.0e15;  // coordinate of the padding slot
__host__ __device__ __forceinline__ int lds_plane(int cap) { return cap + 8; }
// Dynamic LDS of the kernels that stage a tile's region (positions), and of
// those that accumulate over it (three planes of doubles).
__host__ __device__ __forceinline__ size_t lds_region_bytes(int cap) {
    return 3 * sizeof(double) * ((size_t)cap + 1);
}
__host__ __device__ __forceinline__ size_t lds_acc_bytes(int cap) {
    return 3 * sizeof(double) * (size_t)lds_plane(cap);
}

struct RegionBatch {
    static constexpr int R = 10;  // one batch covers most regions (40 chunks, 2 560 slots)
    double4 p[R];
    int4 d[R];
};

__device__ __forceinline__ void region_issue(const Sys& s, const double4* src, int tile, int nchk,
                                             int c0, RegionBatch& b) {
    constexpr int W = kBlock / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int4* chk = s.tile_chunk + (size_t)tile * kChunkMax;
    // every descriptor load first (the index clamped into the tile's table
    // instead of a branch per load, so the loads issue together and are
    // waited for once), then every record load
    const int last = max(nchk - 1, 0);
#pragma unroll
    for (int r = 0; r < RegionBatch::R; r++) b.d[r] = chk[min(c0 + r * W, last)];
#pragma unroll
    for (int r = 0; r < RegionBatch::R; r++) {
        // a chunk past the end re-reads the last one and is not stored (its
        // descriptor still feeds the address, so its load cannot move under
        // a branch); lanes past a chunk's end re-read its last slot
        if (c0 + r * W >= nchk) b.d[r].w = -1;
        b.p[r] = src[b.d[r].x + min(lane, b.d[r].y - b.d[r].x - 1)];
    }
}

__device__ __forceinline__ void region_store(const Sys& s, double* lds, const RegionBatch& b) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int r = 0; r < RegionBatch::R; r++) {
        const int4 d = b.d[r];
        if (d.w >= 0 && lane < d.y - d.x) {
            // the chunk's periodic image is added on the way in
            double* q = lds + 3 * (d.z + lane);
            q[0] = b.p[r].x + (double)((d.w & 3) - 1) * s.box;
            q[1] = b.p[r].y + (double)(((d.w >> 2) & 3) - 1) * s.box;
            q[2] = b.p[r].z + (double)(((d.w >> 4) & 3) - 1) * s.box;
        }
    }
}

// Remaining batches, padding slot and the workgroup barrier.
__device__ __forceinline__ void region_finish(const Sys& s, const double4* src, double* lds,
                                              int cap, int tile, int nchk, int wv,
                                              RegionBatch& rb) {
    constexpr int W = kBlock / kWave;
    for (int c0 = wv + W * RegionBatch::R; c0 < nchk; c0 += W * RegionBatch::R) {
        region_issue(s, src, tile, nchk, c0, rb);
        region_store(s, lds, rb);
    }
    if (threadIdx.x == 0) {
        lds[3 * cap] = kFar;
        lds[3 * cap + 1] = kFar;
        lds[3 * cap + 2] = kFar;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Verlet-list build: one lane per particle, one wavefront per tile (four
// tiles per workgroup).  Each lane appends every j != i with r_ij^2 < r_v^2
// from its 27 neighbour cells to its list, in a fixed order.  For a staged
// tile the wavefront walks the tile's region (the union of its particles'
// neighbourhoods) in FP32 with FP64 deciding inside the rounding band, and
// entries index the region; otherwise every lane gathers its own cells in
// FP64 and stores slots with the minimum-image code.  The build also moves
// the particle records from the reorder buffer back into the state and
// stores the build reference positions; per-tile totals of the half-list
// lengths (entries with j > i) feed the half-list offsets.
// ---------------------------------------------------------------------------

// Exclusive scan of the per-tile half-list totals into tile offsets by one
// workgroup (the last of the list build); records |E|, the longest list, the
// staged tiles and the build count.
__device__ __forceinline__ void scan_tiles(const Sys& s) {
    const long long cap = s.max_half;
    const long long tot = block_scan<16>(
        s.ntiles, [&](int k) { return coh_load(&s.bsum[k]); },
        [&](int k, long long run, int) { s.bsum[k] = (int)(run < cap ? run : cap); });
    __shared__ int rmax[kBlock / kWave], rst[kBlock / kWave];
    int mx = 0, st = 0;
    for (int t = threadIdx.x; t < s.ntiles; t += kBlock) {
        mx = max(mx, coh_load(&s.tmax[t]));
        st += s.tile_nseg[t] >= 0;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off));
        st += __shfl_xor(st, off);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) rmax[threadIdx.x / kWave] = mx, rst[threadIdx.x / kWave] = st;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; w++) mx = max(mx, rmax[w]), st += rst[w];
        s.ctrl->max_count = mx;
        s.ctrl->staged = st;
        s.ctrl->npairs = tot < cap ? tot : cap;
        if (tot > cap) atomicOr(&s.ctrl->overflow, 1);
        s.ctrl->rebuilds += 1;
        s.ctrl->half_stale = 1;
        s.ctrl->eidx_stale = s.estore;
        s.ctrl->rebuild = 0;  // every workgroup of the build has read it
        s.ctrl->req[0] = s.ctrl->req[1] = 0;  // a requested rebuild is done
    }
}

// Pointer into the constant address space: the data does not change while
// the kernel runs, so wavefront-uniform loads through it go to scalar
// registers (one load for the wavefront instead of one per lane).
typedef float cf4 __attribute__((ext_vector_type(4)));
typedef double cd4 __attribute__((ext_vector_type(4)));
typedef int ci4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ const __attribute__((address_space(4))) cf4* as_const(const float4* p) {
    return (const __attribute__((address_space(4))) cf4*)p;
}
__device__ __forceinline__ const __attribute__((address_space(4))) cd4* as_const(const double4* p) {
    return (const __attribute__((address_space(4))) cd4*)p;
}
__device__ __forceinline__ const __attribute__((address_space(4))) ci4* as_const(const int4* p) {
    return (const __attribute__((address_space(4))) ci4*)p;
}

__device__ __forceinline__ void b_build(const Sys& s, int bid, int nb) {
    if (!s.ctrl->rebuild) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int tile = bid * (kBlock / kWave) + __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int i = tile * kTile + lane;
    const bool act = i < s.n;
    const int ii = act ? i : s.n - 1;
    const bool tact = tile < s.ntiles;
    // LJ lists of a tile with a region hold region indices; patchy lists
    // always hold slots (their regions serve the edge pass's accumulator)
    const int nseg = tact && s.pot == 0 ? s.tile_nseg[tile] : -1;
    const double4 xi = s.tpos[ii];
    if (act) {
        s.pos[i] = xi;
        s.xbuild[i] = xi;
        s.vel[i] = s.tvel[i];
        s.id[i] = s.tid[i];
        if (s.pot == 1) {
            s.quat[i] = s.tquat[i];
            s.angm[i] = s.tangm[i];
        }
    }
    const int nc = s.nc;
    const int cx = cell_coord(xi.x, s.cell_inv, nc);
    const int cy = cell_coord(xi.y, s.cell_inv, nc);
    const int cz = cell_coord(xi.z, s.cell_inv, nc);
    // the particle's current row of four entries (slots past n in the last
    // tile have rows of their own, which get the padding)
    int4* wrow = (int4*)list_row_w(s, tact ? i : ii);
    const int cap = s.cap;
    const double rv2 = s.rv2;
    int count = 0, half = 0;
    int e0 = 0, e1 = 0, e2 = 0;  // entries of the current row not yet written
    // staged tile: entry k of the lane's particle is 16-bit word list_off16(k)
    uint16_t* wrow16 = reinterpret_cast<uint16_t*>(list_row_w(s, tact ? i : ii));
    // Appends entry `ent` for partner j; a row of four goes out in one store.
    auto append = [&](int j, int ent) {
        if (count < cap) {
            const int sl = count & 3;
            if (sl == 3) {
                *wrow = make_int4(e0, e1, e2, ent);
                wrow += kTile;
            }
            e0 = sl == 0 ? ent : e0;
            e1 = sl == 1 ? ent : e1;
            e2 = sl == 2 ? ent : e2;
            half += j > i;
        }
        count++;
    };
    // Staged tile: appends region index `reg` for partner j (16-bit entries,
    // stored one by one: the hits of a lane come in a divergent loop, where a
    // store costs less than keeping a row of eight in registers).
    auto append16 = [&](int j, int reg) {
        if (count < cap) {
            wrow16[list_off16(count)] = (uint16_t)reg;
            half += j > i;
        }
        count++;
    };
    if (nseg >= 0) {
        // Staged tile: every lane walks its own 27 cells, row of cells by row
        // (dz, dy) in list order, each row as one run of consecutive slots
        // (cells cx - 1 .. cx + 1), or two where the row wraps the box; the
        // lanes of one home cell read the same records, so a wavefront's
        // load touches a few distinct addresses.  A run lies inside one
        // segment of the tile's region (the segment of the lane's home row
        // for that (dz, dy) and image), which gives the entries' region
        // indices.  The test runs in FP32 on the rounded copy of the records,
        // as t = |x_j - x_i|^2 - lo: t < 0 is in; t >= w (lo + w is the
        // band's top) is out; a candidate with t in [0, w) is decided in
        // FP64, so the list is the one the FP64 test gives.
        const int hr = cz * nc + cy - s.tile_row0[tile];  // the lane's home row in the tile
        const bool inr = act && (unsigned)hr <= 1u;
        const int4* sgp = s.tile_seg + (size_t)tile * kSegMax + (inr ? hr : 0) * 18;
        const float nlo = -s.rv2_lo;
        const unsigned wbits = __float_as_uint(s.rv2_band);
        auto wrapc = [&](int v) { return v < 0 ? 0 : (v >= nc ? 2 : 1); };  // shift -L, 0, +L
        // first cell of the lane's run 0 and the last (run 1 exists only for
        // cx = 0 and cx = nc - 1, where the row wraps the box)
        const int xa0 = cx == 0 ? nc - 1 : cx - 1;
        const int xb0 = cx == 0 ? nc - 1 : (cx == nc - 1 ? nc - 1 : cx + 1);
        const int nrun = __any(inr && (cx == 0 || cx == nc - 1)) ? 2 : 1;
        auto row_of = [&](int r) {  // row of cells (dz, dy) = (r / 3 - 1, r % 3 - 1)
            int az = cz + r / 3 - 1, ay = cy + r % 3 - 1;
            az += az < 0 ? nc : (az >= nc ? -nc : 0);
            ay += ay < 0 ? nc : (ay >= nc ? -nc : 0);
            return (az * nc + ay) * nc;
        };
        // run 0 bounds of the next row, loaded one row ahead
        int ncb = inr ? s.cstart[row_of(0) + xa0] : 0;
        int nce = inr ? s.cstart[row_of(0) + xb0 + 1] : 0;
        for (int r = 0; r < 9; r++) {
            const int dz = r / 3 - 1, dy = r % 3 - 1;
            {
                const int zc = wrapc(cz + dz), yc = wrapc(cy + dy);
                const int rowbase = row_of(r);
                const int cb0 = ncb, ce0 = nce;
                if (r < 8) {
                    ncb = inr ? s.cstart[row_of(r + 1) + xa0] : 0;
                    nce = inr ? s.cstart[row_of(r + 1) + xb0 + 1] : 0;
                }
                const int4 g0 = sgp[r * 2];
                const int4 g1 = sgp[r * 2 + 1];
                for (int run = 0; run < nrun; run++) {
                    // the run's cells [xa, xb] and x image code
                    int xa, xb, xc;
                    if (cx == 0) {
                        xa = run ? 0 : nc - 1, xb = run ? 1 : nc - 1, xc = run ? 1 : 0;
                    } else if (cx == nc - 1) {
                        xa = run ? 0 : nc - 2, xb = run ? 0 : nc - 1, xc = run ? 2 : 1;
                    } else {
                        xa = cx - 1, xb = run ? cx - 2 : cx + 1, xc = 1;  // one run
                    }
                    const bool has = inr && xb >= xa;
                    const int cb = run == 0 ? cb0 : (has ? s.cstart[rowbase + xa] : 0);
                    const int ce = run == 0 ? ce0 : (has ? s.cstart[rowbase + xb + 1] : 0);
                    const int code = xc | yc << 2 | zc << 4;
                    const bool m0 = g0.w == code && cb >= g0.x && cb < g0.y;
                    const bool m1 = g1.w == code && cb >= g1.x && cb < g1.y;
                    const int roff = m0 ? g0.z - g0.x : g1.z - g1.x;  // region index of j: roff + j
                    const int end = (m0 || m1) ? ce : cb;
                    if (ce > cb && !(m0 || m1)) atomicOr(&s.ctrl->overflow, 2);  // region misses the run
                    // x_i in the run's periodic image
                    const double sx = xi.x - (double)(xc - 1) * s.box;
                    const double sy = xi.y - (double)(yc - 1) * s.box;
                    const double sz = xi.z - (double)(zc - 1) * s.box;
                    const float fx = (float)sx, fy = (float)sy, fz = (float)sz;
                    auto tbits = [&](const float4& pf) {
                        const float ex = pf.x - fx, ey = pf.y - fy, ez = pf.z - fz;
                        return __float_as_uint(
                            __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, __builtin_fmaf(ex, ex, nlo))));
                    };
                    // hits collect as bits j - c0 of ma and are appended per
                    // window of 64 candidates (the particle itself and slots
                    // past the run's end are never set)
                    auto flush = [&](int c0, unsigned long long ma) {
                        while (ma) {
                            const int j = c0 + __builtin_ctzll(ma);
                            ma &= ma - 1;
                            append16(j, roff + j);
                        }
                    };
                    // eight candidates per round (reads past the run's end
                    // land in the copy or its spare records); the next
                    // round's records are loaded before this round is tested
                    float4 qn[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) qn[u] = s.tposf[cb + u];
                    unsigned long long ma = 0;
                    int c0 = cb;
                    for (int j0 = cb; j0 < end; j0 += 8) {
                        float4 pv[8];
#pragma unroll
                        for (int u = 0; u < 8; u++) pv[u] = qn[u];
#pragma unroll
                        for (int u = 0; u < 8; u++) qn[u] = s.tposf[j0 + 8 + u];
                        unsigned m8 = 0, tmin = ~0u;
#pragma unroll
                        for (int u = 0; u < 8; u++) {
                            const unsigned tb = tbits(pv[u]);
                            tmin = min(tmin, tb);
                            m8 |= (tb >> 31) << u;
                        }
                        if (tmin < wbits) {  // rare: FP64 decides the candidates in the band
#pragma unroll
                            for (int u = 0; u < 8; u++) {
                                const int j = j0 + u;
                                if (tbits(pv[u]) < wbits && j < end) {
                                    const double4 pj = s.tpos[j];
                                    const double dx = pj.x - sx, dy = pj.y - sy, dz = pj.z - sz;
                                    if (dx * dx + dy * dy + dz * dz < rv2) m8 |= 1u << u;
                                }
                            }
                        }
                        const int left = end - j0;
                        if (left < 8) m8 &= (1u << left) - 1;
                        if ((unsigned)(i - j0) < 8u) m8 &= ~(1u << (i - j0));
                        ma |= (unsigned long long)m8 << (j0 - c0);
                        if (j0 - c0 == 56) {  // a window of 64 is full
                            flush(c0, ma);
                            ma = 0;
                            c0 = j0 + 8;
                        }
                    }
                    flush(c0, ma);
                }
            }
        }
        if (act && (unsigned)hr > 1u) atomicOr(&s.ctrl->overflow, 2);  // region misses the particle
    } else {
        // Global gathers: every lane walks its own 27 cells as runs of
        // consecutive slots (one or two per row of cells; cell by cell when
        // the cells follow a space-filling curve) and stores slot entries
        // with the minimum-image code.
        const int span = nc >= 3 ? 3 : nc;  // distinct cells per dimension
        const int lo = nc >= 3 ? -1 : 0;
        for (int dz = 0; dz < span; dz++) {
            int az = cz + lo + dz;
            az = az < 0 ? az + nc : (az >= nc ? az - nc : az);
            for (int dy = 0; dy < span; dy++) {
                int ay = cy + lo + dy;
                ay = ay < 0 ? ay + nc : (ay >= nc ? ay - nc : ay);
                // The neighbour cells of this row in list order (dx ascending)
                // as runs of consecutive cells: one run (cx - 1 .. cx + 1), or
                // two where the row wraps the box; for nc < 3 every distinct
                // cell on its own.
                int a0, b0, a1 = 0, b1 = 0, nr;
                if (nc >= 3) {
                    if (cx == 0) a0 = b0 = nc - 1, a1 = 0, b1 = 1, nr = 2;
                    else if (cx == nc - 1) a0 = nc - 2, b0 = nc - 1, a1 = b1 = 0, nr = 2;
                    else a0 = cx - 1, b0 = cx + 1, nr = 1;
                } else {
                    a0 = b0 = cx, nr = nc;
                    if (nc == 2) a1 = b1 = 1 - cx;
                }
                const int rowbase = (az * nc + ay) * nc;
                if (s.cell_rank) nr = span;  // one run per cell
                for (int run = 0; run < nr; run++) {
                    int cb, ce;
                    if (s.cell_rank) {
                        int ax = cx + lo + run;
                        ax = ax < 0 ? ax + nc : (ax >= nc ? ax - nc : ax);
                        const int cid = s.cell_rank[rowbase + ax];
                        cb = act ? s.cstart[cid] : 0;
                        ce = act ? s.cstart[cid + 1] : 0;
                    } else {
                        cb = act ? s.cstart[rowbase + (run ? a1 : a0)] : 0;
                        ce = act ? s.cstart[rowbase + (run ? b1 : b0) + 1] : 0;
                    }
                    auto consider = [&](int j, const double4& pj) {
                        const double ex = pj.x - xi.x, ey = pj.y - xi.y, ez = pj.z - xi.z;
                        const double ddx = wrap_delta(ex, s.box, s.inv_box);
                        const double ddy = wrap_delta(ey, s.box, s.inv_box);
                        const double ddz = wrap_delta(ez, s.box, s.inv_box);
                        const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        if (j < ce && j != i && r2 < rv2)
                            append(j, j | (image_code(ex, s.inv_box) | image_code(ey, s.inv_box) << 2 |
                                           image_code(ez, s.inv_box) << 4)
                                              << kSlotBits);
                    };
                    for (int j0 = cb; j0 < ce; j0 += 2) {
                        const double4 p0 = s.tpos[min(j0 + 0, ce - 1)];
                        const double4 p1 = s.tpos[min(j0 + 1, ce - 1)];
                        consider(j0 + 0, p0);
                        consider(j0 + 1, p1);
                    }
                }
            }
        }
    }
    // wavefront (= tile) totals: longest list and half-list length
    int mx = act ? count : 0, hs = act ? half : 0;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off));
        hs += __shfl_xor(hs, off);
    }
    if (nseg >= 0) {
        // Staged tile: every list is padded with the padding slot up to the
        // tile's longest list rounded up to 16 entries, so the vertex pass
        // reads whole rows without masking what lies past a list's end.
        // (A particle's rows hold 8 * mcap >= 16 entries, mcap >= 2.)
        const int bound = min((min(mx, cap) + 15) & ~15, 8 * s.mcap);
        const uint16_t pad = (uint16_t)s.lds_cap;
        if (tact)  // also the rows of slots past n, which the vertex pass reads
            for (int c = min(count, cap); c < bound; c++) wrow16[list_off16(c)] = pad;
    } else if (act && (min(count, cap) & 3)) {  // last, partial row
        *wrow = make_int4(e0, e1, e2, 0);
    }
    if (act) {
        s.ncount[i] = count < cap ? count : cap;
        s.hcount[i] = half;
        if (count > cap) atomicOr(&s.ctrl->overflow, 1);
    }
    if (lane == 0 && tact) {  // read by the last workgroup
        coh_store(&s.tmax[tile], mx);
        coh_store(&s.bsum[tile], hs);
    }
    if (last_block(s.sync + kSyncBuild * kSyncInts, bid, nb)) scan_tiles(s);
}

// At most 128 VGPRs: four wavefronts per SIMD, one full wave of the chip for
// every 1024 tiles.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_build(Sys s) {
    b_build(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}


// Half list (edge and Newton passes), filled on demand after a build: one
// workgroup per tile, four lanes per particle.
// Row starts are the tile offset plus a prefix over the tile's particles; a
// staged tile first maps its LDS indices back to slots (in LDS); each
// particle's lanes walk its full list and keep the entries with j > i,
// compacted with a ballot (list order is kept).  Records the chunk heads
// (first row of every 64-entry chunk) that the edge pass uses.
__device__ __forceinline__ void b_half_fill(const Sys& s, int bid, int nb) {
    if (!s.ctrl->half_stale) return;
    extern __shared__ int map[];
    __shared__ int hpre[kTile];
    constexpr int TPP = kTileTpp;
    const int tile = bid;
    const int i = tile * kTile + threadIdx.x / TPP;
    const int q = threadIdx.x % TPP;
    const int lane = threadIdx.x & (kWave - 1);
    const int gshift = lane & ~(TPP - 1);
    const bool act = i < s.n;
    const int nseg = s.pot == 0 ? s.tile_nseg[tile] : -1;  // region-index lists (LJ)
    // patchy particles whose edge pass goes by tiles: the tile's region, for
    // the region indices of the partners it accumulates over
    const int rseg = s.pot != 0 && patchy_edge_by_tile(s) ? s.tile_nseg[tile] : -1;
    __shared__ int4 sg[kSegMax];
    if (nseg >= 0) {
        const int nchk = s.tile_nchunk[tile];
        const int4* chk = s.tile_chunk + (size_t)tile * kChunkMax;
        for (int c = threadIdx.x / kWave; c < nchk; c += kBlock / kWave) {
            int4 d = chk[c];
            if (lane < d.y - d.x) map[d.z + lane] = (d.x + lane) | d.w << kSlotBits;
        }
    } else if (rseg >= 0 && (int)threadIdx.x < rseg) {
        sg[threadIdx.x] = s.tile_seg[(size_t)tile * kSegMax + threadIdx.x];
    }
    if (threadIdx.x < kTile) {
        int ip = tile * kTile + threadIdx.x;
        hpre[threadIdx.x] = ip < s.n ? s.hcount[ip] : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive prefix over the tile's 64 particles
        int run = 0;
        for (int p = 0; p < kTile; p++) {
            int h = hpre[p];
            hpre[p] = run;
            run += h;
        }
    }
    __syncthreads();
    const long long capl = s.max_half;
    long long start = (long long)s.bsum[tile] + hpre[threadIdx.x / TPP];
    if (start > capl) start = capl;
    const int h = act ? s.hcount[i] : 0;
    long long end = start + h;
    if (end > capl) end = capl;
    if (act && q == 0) {
        s.hstart[i] = (int)start;
        if (i == s.n - 1) s.hstart[s.n] = (int)end;
        for (long long c0 = (start + kWave - 1) / kWave * kWave; c0 < end; c0 += kWave)
            s.chunk_row[c0 / kWave] = i;
    }
    const int cnt = act ? s.ncount[i] : 0;
    const int* row = list_row(s, act ? i : 0);
    const uint16_t* row16 = list_row16(s, act ? i : 0);
    int mine = cnt > q ? (cnt - q + TPP - 1) / TPP : 0;
    int mmax = mine;
    for (int off = kWave / 2; off > 0; off >>= 1) mmax = max(mmax, __shfl_xor(mmax, off));
    long long k = start;
    for (int m = 0; m < mmax; m++) {
        bool ok = m < mine;
        int ent = 0, reg = 0;
        if (ok) {
            if (nseg >= 0) {  // region index -> slot with image
                reg = row16[list_off16(q + m * TPP)];
                ent = map[reg];
            } else {
                ent = row[list_off(q + m * TPP)];
            }
        }
        const int j = entry_slot(ent);
        const bool keep = ok && j > i;
        const unsigned grp = (unsigned)(__ballot(keep) >> gshift) & ((1u << TPP) - 1);
        const long long kk = k + __builtin_popcount(grp & ((1u << q) - 1));
        // deterministic edge mode: entries with j > i are edge kk of this row
        // (the others are filled by the column pass)
        if (s.estore && keep) eidx_row(s, i)[list_off(q + m * TPP)] = kk < end ? (int)kk : -1;
        if (keep && kk < end) {
            s.hj[kk] = ent;
            // the edge pass accumulates by region index and finds the row in
            // the high half (four patches: the region index of slot j in the
            // image of the entry, kNoRegion outside the region)
            if (nseg >= 0) {
                s.hr[kk] = (unsigned)reg | (unsigned)(i - tile * kTile) << 16;
            } else if (rseg >= 0) {
                const int rg = tile_lds_base(sg, rseg, j, (unsigned)ent >> kSlotBits);
                s.hr[kk] = (unsigned)(rg >= 0 ? rg : kNoRegion) | (unsigned)(i - tile * kTile) << 16;
            }
        }
        k += __builtin_popcount(grp);
    }
    // the last workgroup marks the list current (every workgroup has passed
    // its check of the flag by then)
    if (last_block(s.sync + kSyncHalf * kSyncInts, bid, nb) && threadIdx.x == 0) s.ctrl->half_stale = 0;
}

__global__ __launch_bounds__(kBlock) void k_half_fill(Sys s) { b_half_fill(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x); }

// Deterministic edge mode, after the half list: every full-list entry of
// particle i whose partner j is below i gets the index of edge (j, i) in row
// j of the half list, found by a walk over that row, with bit 31 set (i is
// the edge's second member); -1 if the row does not hold it.  One workgroup
// per tile, four lanes per particle, like the half-list fill.
__device__ __forceinline__ void b_col_fill(const Sys& s, int bid, int nb) {
    if (!s.ctrl->eidx_stale) return;
    extern __shared__ int map[];
    constexpr int TPP = kTileTpp;
    const int tile = bid;
    const int i = tile * kTile + threadIdx.x / TPP;
    const int q = threadIdx.x % TPP;
    const int lane = threadIdx.x & (kWave - 1);
    const bool act = i < s.n;
    const int nseg = s.pot == 0 ? s.tile_nseg[tile] : -1;  // region-index lists
    if (nseg >= 0) {
        const int nchk = s.tile_nchunk[tile];
        const int4* chk = s.tile_chunk + (size_t)tile * kChunkMax;
        for (int c = threadIdx.x / kWave; c < nchk; c += kBlock / kWave) {
            int4 d = chk[c];
            if (lane < d.y - d.x) map[d.z + lane] = d.x + lane;
        }
    }
    __syncthreads();
    const int cnt = act ? s.ncount[i] : 0;
    const int* row = list_row(s, act ? i : 0);
    const uint16_t* row16 = list_row16(s, act ? i : 0);
    int* erow = eidx_row(s, act ? i : 0);
    for (int kq = q; kq < cnt; kq += TPP) {
        const int j = nseg >= 0 ? map[row16[list_off16(kq)]] : entry_slot(row[list_off(kq)]);
        if (j >= i) continue;
        int v = -1;
        const int e0 = s.hstart[j], e1 = s.hstart[j + 1];
        // eight entries of row j per round, all loads issued first
        for (int b = e0; b < e1 && v == -1; b += 8) {
            int h[8];
#pragma unroll
            for (int u = 0; u < 8; u++) h[u] = s.hj[min(b + u, e1 - 1)];
#pragma unroll
            for (int u = 7; u >= 0; u--)
                if (b + u < e1 && entry_slot(h[u]) == i) v = (b + u) | INT_MIN;
        }
        erow[list_off(kq)] = v;
    }
    if (last_block(s.sync + kSyncCol * kSyncInts, bid, nb) && threadIdx.x == 0) s.ctrl->eidx_stale = 0;
}

__global__ __launch_bounds__(kBlock) void k_col_fill(Sys s) { b_col_fill(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x); }

// ---------------------------------------------------------------------------
// Vertex decomposition: one thread per particle, no atomics.  Each thread
// walks its own full list, evaluates every pair for itself (each pair is thus
// evaluated twice overall) and writes its own force once.  Optionally fuses
// the closing half kick of velocity Verlet (the particle is owned).
// PREC 0: FP64; 1: FP32 pair maths, FP64 sums; 2: FP32 pair maths, Kahan FP32.
// The cut-off decision is always taken on the FP64 separation.
// ---------------------------------------------------------------------------

template <int PREC>
struct Acc3 {
    double x = 0, y = 0, z = 0;
    __device__ void add(double a, double b, double c) {
        x += a;
        y += b;
        z += c;
    }
    __device__ double gx() const { return x; }
    __device__ double gy() const { return y; }
    __device__ double gz() const { return z; }
};
template <>
struct Acc3<2> {
    float x = 0, y = 0, z = 0, cx = 0, cy = 0, cz = 0;
    __device__ static void k(float& s, float& c, float t) {
        float y = t - c;
        float u = s + y;
        c = (u - s) - y;
        s = u;
    }
    __device__ void add(float a, float b, float c) {
        k(x, cx, a);
        k(y, cy, b);
        k(z, cz, c);
    }
    // compensated value: the running sum minus the carried rounding error
    __device__ double gx() const { return (double)x - (double)cx; }
    __device__ double gy() const { return (double)y - (double)cy; }
    __device__ double gz() const { return (double)z - (double)cz; }
};

#ifndef MD_VERTEX_TPP
#define MD_VERTEX_TPP 1
#endif
#ifndef MD_VERTEX_UNROLL
#define MD_VERTEX_UNROLL 4
#endif
constexpr int kVertexTpp = MD_VERTEX_TPP;        // lanes per particle, LJ vertex pass
constexpr int kVertexUnroll = MD_VERTEX_UNROLL;  // gathers in flight per lane

// One list entry of the LJ vertex pass.  Branch-free: entries beyond r_c
// contribute an exact zero.  The separation is formed in FP64, with the
// entry's stored image (global gathers) or from an LDS copy that already
// carries the image (PRESHIFTED); PREC > 0 does the rest in FP32.
template <int PREC, bool ENERGY, bool PRESHIFTED = false>
__device__ __forceinline__ void lj_vertex_term(const Sys& s, const double4& xi, int ent,
                                               const double4& xj, Acc3<PREC>& f, double& e,
                                               double& w) {
    double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
    if (!PRESHIFTED) {
        dx += image(ent, 0, s.box);
        dy += image(ent, 1, s.box);
        dz += image(ent, 2, s.box);
    }
    double r2 = dx * dx + dy * dy + dz * dz;
    bool in = r2 < s.rc2;
    if (PREC == 0) {
        double inv = rcp_nr(r2);
        double s2 = s.l64.sig2 * inv;
        double s6 = s2 * s2 * s2;
        double fr = in ? s.l64.eps24 * inv * s6 * (2.0 * s6 - 1.0) : 0.0;
        f.add(-fr * dx, -fr * dy, -fr * dz);
        if (ENERGY && in) {
            e += 0.5 * (s.l64.eps4 * s6 * (s6 - 1.0) - s.l64.vshift);
            w += 0.5 * fr * r2;
        }
    } else {
        float r2f = (float)r2;
        float inv = rcp_nr(r2f);
        float s2 = s.l32.sig2 * inv;
        float s6 = s2 * s2 * s2;
        float fr = in ? s.l32.eps24 * inv * s6 * (2.0f * s6 - 1.0f) : 0.0f;
        f.add(-fr * (float)dx, -fr * (float)dy, -fr * (float)dz);
        if (ENERGY && in) {
            e += 0.5 * (double)(s.l32.eps4 * s6 * (s6 - 1.0f) - s.l32.vshift);
            w += 0.5 * (double)fr * r2;
        }
    }
}

// TPP lanes share particle i and take every TPP-th list entry; each lane
// keeps kVertexUnroll independent gathers in flight; the TPP partial sums are
// combined with cross-lane shuffles before the single owner write.
// Walks entries q, q + TPP, ... of particle i's list with global gathers
// (tiles whose region was not staged).
template <int PREC, int TPP, bool ENERGY>
__device__ __forceinline__ void lj_walk_global(const Sys& s, int ii, int q, int cnt,
                                               const double4& xi, Acc3<PREC>& f, double& e,
                                               double& w) {
    constexpr int U = kVertexUnroll;
    const int* nb = list_row(s, ii);
    int k = q;
    for (; k + (U - 1) * TPP < cnt; k += U * TPP) {
        int en[U];
        double4 xj[U];
#pragma unroll
        for (int u = 0; u < U; u++) en[u] = __builtin_nontemporal_load(nb + list_off(k + u * TPP));
#pragma unroll
        for (int u = 0; u < U; u++) xj[u] = s.pos[entry_slot(en[u])];
#pragma unroll
        for (int u = 0; u < U; u++) lj_vertex_term<PREC, ENERGY>(s, xi, en[u], xj[u], f, e, w);
    }
    for (; k < cnt; k += TPP) {
        int en = __builtin_nontemporal_load(nb + list_off(k));
        lj_vertex_term<PREC, ENERGY>(s, xi, en, s.pos[entry_slot(en)], f, e, w);
    }
}

#ifndef MD_VERTEX_PREFETCH
#define MD_VERTEX_PREFETCH 24
#endif
constexpr int kPrefetch = MD_VERTEX_PREFETCH;  // list entries held in registers per lane

// F/r of the LJ pair at separation^2 r2, exactly zero from r_c on: there the
// high word of r2 is replaced by that of 1e300 (FP64; 1e30 in FP32), whose
// inverse cubed underflows to zero.  F/r = r^-2 u (c12 u - c6), u = r^-6.
__device__ __forceinline__ double lj_fr_cut(const Sys& s, double r2) {
    const bool in = r2 < s.rc2;
    const double r2m = __hiloint2double(in ? __double2hiint(r2) : 0x7E37E43C, __double2loint(r2));
    const double inv = rcp_nr(r2m);
    const double u = inv * inv * inv;
    return inv * u * fma(s.l64.c12, u, -s.l64.c6);
}
__device__ __forceinline__ float lj_fr_cut32(const Sys& s, double r2) {
    const float r2f = r2 < s.rc2 ? (float)r2 : 1e30f;
    const float inv = rcp_nr(r2f);
    const float u = inv * inv * inv;
    return inv * u * fmaf(s.l32.c12, u, -s.l32.c6);
}

// Branch-free LJ term from an LDS image that already carries the periodic
// image.  The cut-off selects a 0/1 factor, so every lane runs the same
// instruction stream.
template <int PREC, bool ENERGY>
__device__ __forceinline__ void lj_pos_term(const Sys& s, double px, double py, double pz,
                                            const double4& xi, Acc3<PREC>& f, double& e,
                                            double& w) {
    double dx = px - xi.x;
    double dy = py - xi.y;
    double dz = pz - xi.z;
    double r2 = dx * dx + dy * dy + dz * dz;
    if (!ENERGY) {
        if (PREC == 0) {
            const double fr = lj_fr_cut(s, r2);
            f.add(-fr * dx, -fr * dy, -fr * dz);
        } else {
            const float fr = lj_fr_cut32(s, r2);
            f.add(-fr * (float)dx, -fr * (float)dy, -fr * (float)dz);
        }
        return;
    }
    bool in = r2 < s.rc2;
    if (PREC == 0) {
        double inv = rcp_nr(r2);
        double s2 = s.l64.sig2 * inv;
        double s6 = s2 * s2 * s2;
        double fr = s.l64.eps24 * inv * s6 * (2.0 * s6 - 1.0) * (in ? 1.0 : 0.0);
        f.add(-fr * dx, -fr * dy, -fr * dz);
        if (ENERGY && in) {
            e += 0.5 * (s.l64.eps4 * s6 * (s6 - 1.0) - s.l64.vshift);
            w += 0.5 * fr * r2;
        }
    } else {
        float r2f = (float)r2;
        float inv = rcp_nr(r2f);
        float s2 = s.l32.sig2 * inv;
        float s6 = s2 * s2 * s2;
        float fr = s.l32.eps24 * inv * s6 * (2.0f * s6 - 1.0f) * (in ? 1.0f : 0.0f);
        f.add(-fr * (float)dx, -fr * (float)dy, -fr * (float)dz);
        if (ENERGY && in) {
            e += 0.5 * (double)(s.l32.eps4 * s6 * (s6 - 1.0f) - s.l32.vshift);
            w += 0.5 * (double)fr * r2;
        }
    }
}

// One workgroup per tile of kTile particles, TPP = kBlock / kTile lanes per
// particle (in a staged tile lane q of particle i takes entries 2q, 2q + 1,
// 2q + 8, 2q + 9, ...; otherwise q, q + TPP, ...).  A staged tile requests the
// lane's first kPrefetch list entries, copies its region
// into LDS meanwhile, then evaluates the entries from LDS in groups of four
// under a wave-uniform trip count (entries past the list end point at the
// padding slot).  Unstaged tiles gather from global memory.
// DRIFT (with KICK): after the closing half kick, also the next step's half
// kick and drift, written to the other position buffer (pos_alt) because the
// neighbours still read pos, and the next step's rebuild test; the same
// arithmetic as k_kick followed by k_kick_drift.
template <int PREC, int TPP, bool KICK, bool ENERGY, bool DRIFT = false>
__device__ __forceinline__ void b_vertex_lj(const Sys& s, int bid, int nb) {
    static_assert(TPP * kTile == kBlock, "one tile per workgroup");
    static_assert(kPrefetch % 4 == 0, "groups of four");
    static_assert(!DRIFT || KICK, "the drift follows the closing kick");
    extern __shared__ double lds3[];
    const int tile = bid;
    if (DRIFT) {
        // a rebuild requested by the previous launch's drift (or passed on by
        // a launch that did nothing for it): this launch does nothing either
        const int prev = s.launch_id - 1;
        if (s.ctrl->req[prev & 1] == prev) {
            if (bid == 0 && threadIdx.x == 0) s.ctrl->req[s.launch_id & 1] = s.launch_id;
            return;
        }
        if (bid == 0 && threadIdx.x == 0)
            __hip_atomic_store(s.host_run, s.launch_id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    const int i = tile * kTile + threadIdx.x / TPP;
    const int q = threadIdx.x % TPP;
    const int nseg = s.tile_nseg[tile];
    const int cap = s.lds_cap;
    bool act = i < s.n;
    int ii = act ? i : s.n - 1;  // idle lanes stay for the group shuffle
    double4 xi = s.pos[ii];
    int cnt = act ? s.ncount[ii] : 0;
    // the kick's and drift's own loads, issued now so that the epilogue does
    // not wait for memory
    double4 vi = make_double4(0, 0, 0, 0), xb = make_double4(0, 0, 0, 0);
    if (KICK && act && q == 0) vi = s.vel[i];
    if (DRIFT && act && q == 0) xb = s.xbuild[i];
    Acc3<PREC> f;
    double e = 0, w = 0;
    if (nseg >= 0) {
        constexpr int E = kPrefetch;
        // lane entry n is list entry 8 (n / 2) + 2 q + n % 2 (16-bit entries,
        // two per 32-bit word, four words per row of a particle)
        const int mine = 2 * (cnt >> 3) + min(max((cnt & 7) - 2 * q, 0), 2);  // entries of this lane
        int mmax = mine;
        for (int off = kWave / 2; off > 0; off >>= 1) mmax = max(mmax, __shfl_xor(mmax, off));
        mmax = __builtin_amdgcn_readfirstlane(mmax);
        // region copy, first batch: issued before the list prefetch
        const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        const int nchk = s.tile_nchunk[tile];
        RegionBatch rb;
        region_issue(s, s.pos, tile, nchk, wv, rb);
        // The word of lane entries n, n + 1 (n even) in row n / 2 sits at
        // int offset 256 (n / 2) + threadIdx.x of the tile's rows, so a block
        // of E entries is one lane base plus constant offsets.  Every lane
        // issues the loads of the words below the wavefront's longest lane
        // list (a wave-uniform test; the list allocation has kListPadRows
        // spare rows after the last tile); entries past the lane's own list
        // end become the padding slot.
        static_assert(TPP == 4 && kTile * TPP == kBlock, "word offset 256 m + tid");
        static_assert(E % 2 == 0 && E / 2 <= kListPadRows, "prefetch beyond the spare rows");
        const int* lane_rows = s.nbr + (size_t)tile * s.mcap * (kTile * 4) + threadIdx.x;
        // The list build pads a staged tile's lists with the padding slot up
        // to the tile's longest list rounded up to 16 entries, which covers
        // every group of four lane entries below mmax: no masking here.
        // The words stay packed (two entries each) until they are used.
        auto load_block = [&](int n0, unsigned (&wd)[E / 2]) {
            const int* bp = lane_rows + (size_t)(n0 >> 1) * (kTile * 4);
#pragma unroll
            for (int m = 0; m < E / 2; m++) {
                if (n0 + 2 * m < mmax) wd[m] = (unsigned)__builtin_nontemporal_load(bp + m * (kTile * 4));
                else wd[m] = 0u;  // never evaluated
            }
        };
        // groups of four: the four records are read from LDS before the
        // first is used, so their latencies overlap
        auto eval_block = [&](int m0, const unsigned (&wd)[E / 2]) {
#pragma unroll
            for (int m = 0; m < E; m += 4) {
                if (m0 + m < mmax) {
                    double px[4], py[4], pz[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const unsigned w = wd[(m + u) >> 1];
                        const unsigned a = 3u * ((m + u) & 1 ? w >> 16 : w & 0xffffu);
                        px[u] = lds3[a];
                        py[u] = lds3[a + 1];
                        pz[u] = lds3[a + 2];
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) lj_pos_term<PREC, ENERGY>(s, px[u], py[u], pz[u], xi, f, e, w);
                }
            }
        };
        unsigned ea[E / 2], eb[E / 2];
        load_block(0, ea);
        region_store(s, lds3, rb);
        region_finish(s, s.pos, lds3, cap, tile, nchk, wv, rb);
        // long lists: blocks of E entries, the next block's loads in flight
        // while the current one is evaluated
        for (int m0 = 0; m0 < mmax; m0 += 2 * E) {
            if (m0 + E < mmax) load_block(m0 + E, eb);
            eval_block(m0, ea);
            if (m0 + E < mmax) {
                if (m0 + 2 * E < mmax) load_block(m0 + 2 * E, ea);
                eval_block(m0 + E, eb);
            }
        }
    } else {
        lj_walk_global<PREC, TPP, ENERGY>(s, ii, q, cnt, xi, f, e, w);
    }
    double fx = f.gx(), fy = f.gy(), fz = f.gz();
#pragma unroll
    for (int off = TPP / 2; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
        if (ENERGY) {
            e += __shfl_xor(e, off);
            w += __shfl_xor(w, off);
        }
    }
    if (!act || q != 0) return;
    if (ENERGY) {  // energy pass: leaves the forces of the last force pass alone
        s.epart[i] = e;
        s.wpart[i] = w;
        return;
    }
    // The fused step (DRIFT) keeps its forces in registers: nothing reads
    // them before the next force pass (the last step of md_step is never a
    // fused one and stores them).
    if (!DRIFT) s.frc[i] = make_double4(fx, fy, fz, 0.0);
    if (!isfinite(fx + fy + fz)) atomicOr(&s.ctrl->nonfinite, 1);
    if (KICK) {
        double4 v = vi;
        v.x += s.hdt * fx * s.inv_mass;
        v.y += s.hdt * fy * s.inv_mass;
        v.z += s.hdt * fz * s.inv_mass;
        if (DRIFT) {
            v.x += s.hdt * fx * s.inv_mass;
            v.y += s.hdt * fy * s.inv_mass;
            v.z += s.hdt * fz * s.inv_mass;
            double4 x = xi;
            x.x += s.dt * v.x;  // unwrapped until the next list build
            x.y += s.dt * v.y;
            x.z += s.dt * v.z;
            s.pos_alt[i] = x;
            const double ddx = x.x - xb.x, ddy = x.y - xb.y, ddz = x.z - xb.z;
            if (ddx * ddx + ddy * ddy + ddz * ddz > s.disp2) {
                s.ctrl->rebuild = 1;
                s.ctrl->req[s.launch_id & 1] = s.launch_id;
            }
        }
        s.vel[i] = v;
    }
}

// The staged region limits the pass to four workgroups (four waves per SIMD)
// per CU; at most 128 VGPRs keep all four resident.
template <int PREC, int TPP, bool KICK, bool ENERGY, bool DRIFT = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_vertex_lj(Sys s) {
    b_vertex_lj<PREC, TPP, KICK, ENERGY, DRIFT>(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

template <int PREC, bool KICK, bool ENERGY, int TPP>
__device__ __forceinline__ void b_vertex_patchy(const Sys& s, int bid, int nb) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    // TPP lanes per particle: lane q takes list entries q, q + TPP, ...; the
    // partial sums are then combined across the particle's lanes (a fixed
    // order: deterministic).  Several lanes per particle pay where one lane
    // per particle leaves the chip idle (small systems, patchy_vertex_tpp).
    const int i = bid * (kBlock / TPP) + (int)threadIdx.x / TPP;
    const int q = (int)threadIdx.x % TPP;
    if (KICK && bid == 0 && threadIdx.x == 0) s.ctrl->rebuild = 0;
    const bool act = i < s.n;
    const int ii = act ? i : s.n - 1;
    double4 xi = s.pos[ii];
    V3<double> ui[4];
    patch_dirs<double>(s.quat[ii], ui, s.p64.model);
    int cnt = act ? s.ncount[i] : 0;
    Acc3<PREC> f, t;
    double e = 0, w = 0;
    const int* row = list_row(s, ii);
    for (int k = q; k < cnt; k += TPP) {
        int ent = row[list_off(k)];
        int j = entry_slot(ent);
        double4 xj = s.pos[j];
        double dx = xj.x - xi.x + image(ent, 0, s.box);
        double dy = xj.y - xi.y + image(ent, 1, s.box);
        double dz = xj.z - xi.z + image(ent, 2, s.box);
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < s.rc2) {
            V3<double> uj[4];
            patch_dirs<double>(s.quat[j], uj, s.p64.model);
            V3<double> d = {dx, dy, dz};
            V3<double> fj, ti, tj;
            double v;
            patchy_pair<R>(d, r2, ui, uj, s, fj, ti, tj, v);
            f.add(-fj.x, -fj.y, -fj.z);
            t.add(ti.x, ti.y, ti.z);
            if (ENERGY) {
                e += 0.5 * (double)v;
                w += 0.5 * ((double)fj.x * dx + (double)fj.y * dy + (double)fj.z * dz);
            }
        }
    }
    double fx = f.gx(), fy = f.gy(), fz = f.gz();
    double tx = t.gx(), ty = t.gy(), tz = t.gz();
#pragma unroll
    for (int off = 1; off < TPP; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
        tx += __shfl_xor(tx, off);
        ty += __shfl_xor(ty, off);
        tz += __shfl_xor(tz, off);
        if (ENERGY) {
            e += __shfl_xor(e, off);
            w += __shfl_xor(w, off);
        }
    }
    if (!act || q != 0) return;
    if (ENERGY) {
        s.epart[i] = e;
        s.wpart[i] = w;
        return;
    }
    s.frc[i] = make_double4(fx, fy, fz, 0.0);
    s.trq[i] = make_double4(tx, ty, tz, 0.0);
    if (!isfinite(fx + fy + fz + tx + ty + tz)) atomicOr(&s.ctrl->nonfinite, 1);
    if (KICK) {
        double4 v = s.vel[i];
        v.x += s.hdt * fx * s.inv_mass;
        v.y += s.hdt * fy * s.inv_mass;
        v.z += s.hdt * fz * s.inv_mass;
        s.vel[i] = v;
        double4 L = s.angm[i];
        L.x += s.hdt * tx;
        L.y += s.hdt * ty;
        L.z += s.hdt * tz;
        s.angm[i] = L;
    }
}

template <int PREC, bool KICK, bool ENERGY, int TPP>
__global__ __launch_bounds__(kBlock) void k_vertex_patchy(Sys s) {
    b_vertex_patchy<PREC, KICK, ENERGY, TPP>(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// ---------------------------------------------------------------------------
// Edge decomposition: one lane per half-list entry (pair i < j).  The lane
// evaluates the pair once; if the result is exactly zero it writes nothing,
// otherwise it adds -F (and tau_i) to i and +F (and tau_j) to j.  Entries are
// sorted by row, so lanes of a wave that share i first combine their i-side
// terms with a segmented shuffle reduction and one lane per row issues the
// atomics; the j side is one hardware FP64 atomic per component.
// Forces (and torques) must be zero on entry.
// ---------------------------------------------------------------------------

template <typename R>
struct EdgeOut {
    double fx, fy, fz;       // force on j (force on i is minus this)
    double tix, tiy, tiz;    // torque on i
    double tjx, tjy, tjz;    // torque on j
};

// Segmented suffix sum over lanes with equal key (keys ascending with lane);
// afterwards the first lane of each run holds the run's total.
__device__ __forceinline__ double seg_sum(double v, int key, int lane) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        double o = __shfl_down(v, off);
        int ok = __shfl_down(key, off);
        if (lane + off < kWave && ok == key) v += o;
    }
    return v;
}

// STORE (deterministic edge mode): no atomics; every edge's results go to
// the per-edge arrays (zeros included) for the gather pass.
template <int POT, int PREC, bool STORE = false>
__device__ __forceinline__ void b_edge(const Sys& s, int bid, int nb) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    const long long npairs = s.ctrl->npairs;
    const long long nchunks = (npairs + kWave - 1) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const long long nw = (long long)nb * (kBlock / kWave);
    const long long w0 = (long long)bid * (kBlock / kWave) +
                         threadIdx.x / kWave;
    double* F = reinterpret_cast<double*>(s.frc);
    double* T = reinterpret_cast<double*>(s.trq);
    for (long long m = w0; m < nchunks; m += nw) {
        const int r0 = s.chunk_row[m];
        const int rlast = (m + 1 < nchunks) ? s.chunk_row[m + 1] : s.n - 1;
        const long long e = m * kWave + lane;
        const bool valid = e < npairs;
        // row of entry e: the last row in [r0, rlast] whose start is <= e
        int row = r0;
        if (rlast - r0 <= kWave) {
            // dense half list: one coalesced load of the chunk's row starts,
            // counted through lane reads
            int rr = r0 + 1 + lane;
            int hs = rr <= rlast ? s.hstart[rr] : INT_MAX;
            int lim = rlast - r0;
            for (int q = 0; q < lim; q++) row += (__builtin_amdgcn_readlane(hs, q) <= e);
        } else {
            // sparse half list (a chunk spans many rows, most of them empty):
            // binary search per lane
            int lo = r0, hi = rlast;
            while (lo < hi) {
                const int mid = lo + (hi - lo + 1) / 2;
                if ((long long)s.hstart[mid] <= e) lo = mid;
                else hi = mid - 1;
            }
            row = lo;
        }
        const int i = row;
        const int ent = valid ? s.hj[e] : i;
        const int j = min(entry_slot(ent), s.n - 1);
        double fx = 0, fy = 0, fz = 0, tix = 0, tiy = 0, tiz = 0, tjx = 0, tjy = 0, tjz = 0;
        if (valid) {
            double4 xi = s.pos[i], xj = s.pos[j];
            double dx = xj.x - xi.x + image(ent, 0, s.box);
            double dy = xj.y - xi.y + image(ent, 1, s.box);
            double dz = xj.z - xi.z + image(ent, 2, s.box);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < s.rc2) {
                if (POT == 0) {
                    if (PREC == 0) {
                        double fr = lj_fr<double>(r2, s.l64, nullptr);
                        fx = fr * dx;
                        fy = fr * dy;
                        fz = fr * dz;
                    } else {
                        float fr = lj_fr<float>((float)r2, s.l32, nullptr);
                        fx = fr * (float)dx;
                        fy = fr * (float)dy;
                        fz = fr * (float)dz;
                    }
                } else {
                    V3<double> ui[4], uj[4];
                    patch_dirs<double>(s.quat[i], ui, s.p64.model);
                    patch_dirs<double>(s.quat[j], uj, s.p64.model);
                    V3<double> d = {dx, dy, dz};
                    V3<double> fj, ti, tj;
                    double v;
                    patchy_pair<R>(d, r2, ui, uj, s, fj, ti, tj, v);
                    fx = fj.x;
                    fy = fj.y;
                    fz = fj.z;
                    tix = ti.x;
                    tiy = ti.y;
                    tiz = ti.z;
                    tjx = tj.x;
                    tjy = tj.y;
                    tjz = tj.z;
                }
            }
        }
        if (STORE) {
            if (valid) {
                constexpr int C = POT == 1 ? 3 : 1;  // records per edge
                double4* ef = s.ef + (size_t)e * C;
                ef[0] = make_double4(fx, fy, fz, 0.0);
                if (POT == 1) {
                    ef[1] = make_double4(tix, tiy, tiz, 0.0);
                    ef[2] = make_double4(tjx, tjy, tjz, 0.0);
                }
            }
            continue;
        }
        const bool fnz = (fx != 0.0) | (fy != 0.0) | (fz != 0.0);
        const bool tjnz = (tjx != 0.0) | (tjy != 0.0) | (tjz != 0.0);
        const bool nz = fnz | tjnz | (tix != 0.0) | (tiy != 0.0) | (tiz != 0.0);
        // j side: only non-zero results touch memory (a pair inside the core
        // range with no patch in reach has a force but no torques)
        if (fnz) {
            unsafeAtomicAdd(F + 4 * (size_t)j + 0, fx);
            unsafeAtomicAdd(F + 4 * (size_t)j + 1, fy);
            unsafeAtomicAdd(F + 4 * (size_t)j + 2, fz);
        }
        if (POT == 1 && tjnz) {
            unsafeAtomicAdd(T + 4 * (size_t)j + 0, tjx);
            unsafeAtomicAdd(T + 4 * (size_t)j + 1, tjy);
            unsafeAtomicAdd(T + 4 * (size_t)j + 2, tjz);
        }
        // i side: combine the lanes of each row, skip all-zero rows
        const int key = valid ? i : s.n + lane;
        const bool anynz = __any(nz);
        if (anynz) {
            double sx = seg_sum(-fx, key, lane);
            double sy = seg_sum(-fy, key, lane);
            double sz = seg_sum(-fz, key, lane);
            double ux = 0, uy = 0, uz = 0;
            if (POT == 1) {
                ux = seg_sum(tix, key, lane);
                uy = seg_sum(tiy, key, lane);
                uz = seg_sum(tiz, key, lane);
            }
            int up = __shfl_up(key, 1);
            bool head = valid && (lane == 0 || up != key);
            const bool rfnz = (sx != 0.0) | (sy != 0.0) | (sz != 0.0);
            const bool rtnz = (ux != 0.0) | (uy != 0.0) | (uz != 0.0);
            if (head && rfnz) {
                unsafeAtomicAdd(F + 4 * (size_t)i + 0, sx);
                unsafeAtomicAdd(F + 4 * (size_t)i + 1, sy);
                unsafeAtomicAdd(F + 4 * (size_t)i + 2, sz);
            }
            if (POT == 1 && head && rtnz) {
                unsafeAtomicAdd(T + 4 * (size_t)i + 0, ux);
                unsafeAtomicAdd(T + 4 * (size_t)i + 1, uy);
                unsafeAtomicAdd(T + 4 * (size_t)i + 2, uz);
            }
        }
    }
}

template <int POT, int PREC, bool STORE = false>
__global__ __launch_bounds__(kBlock) void k_edge(Sys s) {
    b_edge<POT, PREC, STORE>(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// Half-list entries whose pair result (the force, or for patchy particles
// either torque) is non-zero at the current positions, evaluated in the
// system's precision: the pairs whose atomics the edge pass does not skip
// (Methods section: only non-zero interactions are written).  One thread per
// entry, its row by binary search over the row starts; one 64-bit atomic per
// wavefront into ctrl->nonzero.  Counting only: no force is written.
template <int POT, int PREC>
__global__ __launch_bounds__(kBlock) void k_count_nonzero(Sys s) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    const long long npairs = s.ctrl->npairs;
    unsigned long long cnt = 0;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < npairs;
         e += (long long)gridDim.x * kBlock) {
        int lo = 0, hi = s.n - 1;  // last row whose start is <= e
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if ((long long)s.hstart[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int ent = s.hj[e];
        const int j = min(entry_slot(ent), s.n - 1);
        const double4 xi = s.pos[lo], xj = s.pos[j];
        const double dx = xj.x - xi.x + image(ent, 0, s.box);
        const double dy = xj.y - xi.y + image(ent, 1, s.box);
        const double dz = xj.z - xi.z + image(ent, 2, s.box);
        const double r2 = dx * dx + dy * dy + dz * dz;
        bool nz = false;
        if (r2 < s.rc2) {
            if (POT == 0) {
                const R fr = PREC == 0 ? (R)lj_fr<double>(r2, s.l64, nullptr)
                                       : (R)lj_fr<float>((float)r2, s.l32, nullptr);
                nz = ((R)dx * fr != R(0)) | ((R)dy * fr != R(0)) | ((R)dz * fr != R(0));
            } else {
                V3<double> ui[4], uj[4];
                patch_dirs<double>(s.quat[lo], ui, s.p64.model);
                patch_dirs<double>(s.quat[j], uj, s.p64.model);
                const V3<double> d = {dx, dy, dz};
                V3<double> fj, ti, tj;
                double v;
                patchy_pair<R>(d, r2, ui, uj, s, fj, ti, tj, v);
                nz = (fj.x != 0.0) | (fj.y != 0.0) | (fj.z != 0.0) | (ti.x != 0.0) |
                     (ti.y != 0.0) | (ti.z != 0.0) | (tj.x != 0.0) | (tj.y != 0.0) | (tj.z != 0.0);
            }
        }
        cnt += nz ? 1u : 0u;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & (kWave - 1)) == 0 && cnt)
        atomicAdd(reinterpret_cast<unsigned long long*>(&s.ctrl->nonzero), cnt);
}

__global__ void k_zero_nonzero(Ctrl* c) { c->nonzero = 0; }

// Deterministic edge mode, second pass: four lanes per particle sum the
// stored results of its edges (-F as the edge's first member, +F as its
// second; tau_i or tau_j), lane q the entries q, q + 4, ... of its list in
// order, then the four partial sums in a fixed order, so the forces do not
// depend on scheduling.  Writes F (and tau) for the closing kick.
template <int POT>
__device__ __forceinline__ void b_edge_gather(const Sys& s, int bid, int nb) {
    constexpr int TPP = kTileTpp, U = 4, C = POT == 1 ? 3 : 1;
    const int i = bid * kTile + threadIdx.x / TPP;
    const int q = threadIdx.x % TPP;
    const bool act = i < s.n;
    const int ii = act ? i : s.n - 1;
    const int cnt = act ? s.ncount[ii] : 0;
    const int* erow = eidx_row(s, ii);
    double fx = 0, fy = 0, fz = 0, tx = 0, ty = 0, tz = 0;
    for (int k0 = q; k0 < cnt; k0 += U * TPP) {
        int v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int kk = k0 + u * TPP;
            v[u] = kk < cnt ? erow[list_off(kk)] : -1;
        }
        double4 fe[U], te[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const size_t e = (size_t)(v[u] == -1 ? 0 : (v[u] & INT_MAX));
            fe[u] = s.ef[e * C];
            if (POT == 1) te[u] = s.ef[e * C + (v[u] < 0 ? 2 : 1)];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (v[u] == -1) continue;
            const double g = v[u] < 0 ? 1.0 : -1.0;
            fx += g * fe[u].x;
            fy += g * fe[u].y;
            fz += g * fe[u].z;
            if (POT == 1) {
                tx += te[u].x;
                ty += te[u].y;
                tz += te[u].z;
            }
        }
    }
#pragma unroll
    for (int off = 1; off < TPP; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
        if (POT == 1) {
            tx += __shfl_xor(tx, off);
            ty += __shfl_xor(ty, off);
            tz += __shfl_xor(tz, off);
        }
    }
    if (!act || q != 0) return;
    s.frc[i] = make_double4(fx, fy, fz, 0.0);
    if (POT == 1) s.trq[i] = make_double4(tx, ty, tz, 0.0);
    if (!isfinite(fx + fy + fz + tx + ty + tz)) atomicOr(&s.ctrl->nonfinite, 1);
}

template <int POT>
__global__ __launch_bounds__(kBlock) void k_edge_gather(Sys s) { b_edge_gather<POT>(s, blockIdx.x, gridDim.x); }

// Adds a staged tile's region accumulator (three planes, like the staged
// positions) to global memory: one atomic per non-zero component, the
// region's slots in runs of consecutive slots (one wavefront per run).
// Component c of slot k is dst[c * cstride + k * sstride]: the records of F
// (cstride 1, sstride 4) or the force planes (cstride s.fps, sstride 1).
__device__ __forceinline__ void region_acc_flush(const Sys& s, const double* acc, int plane,
                                                 int tile, double* dst, size_t cstride = 1,
                                                 int sstride = 4) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nchk = s.tile_nchunk[tile];
    const int4* chk = s.tile_chunk + (size_t)tile * kChunkMax;
    for (int c = threadIdx.x / kWave; c < nchk; c += kBlock / kWave) {
        const int4 d = chk[c];
        if (lane < d.y - d.x) {
            const int r = d.z + lane;
            const double vx = acc[r], vy = acc[plane + r], vz = acc[2 * plane + r];
            if ((vx != 0.0) | (vy != 0.0) | (vz != 0.0)) {
                double* g = dst + (size_t)sstride * (size_t)(d.x + lane);
                unsafeAtomicAdd(g, vx);
                unsafeAtomicAdd(g + cstride, vy);
                unsafeAtomicAdd(g + 2 * cstride, vz);
            }
        }
    }
}

// LJ edge pass, one workgroup per tile of kTile rows (the rows' half-list
// entries are contiguous, in row order).
//
// Tiles with a staged region (b_edge_lj_staged): the region's positions are
// copied into LDS as the vertex pass copies them, and each lane takes four
// consecutive half-list entries with one 16-byte load of their packed words
// (row in the tile << 16 | region index of the partner): no global gather
// and no search for the row.  Each pair is evaluated once; the partner's
// share goes into an LDS accumulator over the region with LDS atomics, the
// row's share is summed in registers over the lane's run of entries of one
// row and added to a per-row LDS accumulator once per run.  At the end every
// non-zero accumulator is added to global memory with one atomic per
// component (the region in runs of consecutive slots).  Zero results are
// skipped throughout.  The pass adds into the force planes (x, y and z in
// arrays of their own, so the atomics of a run of slots are 8 bytes apart);
// the closing kick, or k_forces_from_planes, gives the force records.
//
// Other tiles (b_edge_lj_gather): one entry per lane, positions gathered from
// global memory, the row found by binary search over the tile's row starts,
// the partner's share added with global atomics, the row's share combined by
// a segmented shuffle reduction.  The force planes must be zero on entry.

// Dynamic LDS of the LJ edge pass: with staged positions the region copy and
// its accumulator, else the accumulator alone (regions too large for both
// run every tile through the gather path).
constexpr int kEdgeStageCapMax = 3072;
__host__ __device__ constexpr bool edge_stages_positions(int cap) { return cap <= kEdgeStageCapMax; }
__host__ __device__ __forceinline__ size_t edge_lds_bytes(int cap) {
    return (edge_stages_positions(cap) ? lds_region_bytes(cap) : 0) + lds_acc_bytes(cap);
}

// Adds the per-row sums of an LJ edge tile (three doubles per row) to the
// force planes, one atomic per non-zero component.
__device__ __forceinline__ void edge_rows_flush(const Sys& s, const double* fi, int t0, int nrow) {
    if (threadIdx.x < nrow) {
        const double vx = fi[3 * threadIdx.x], vy = fi[3 * threadIdx.x + 1],
                     vz = fi[3 * threadIdx.x + 2];
        if ((vx != 0.0) | (vy != 0.0) | (vz != 0.0)) {
            double* g = s.fpl + (size_t)(t0 + threadIdx.x);
            unsafeAtomicAdd(g, vx);
            unsafeAtomicAdd(g + s.fps, vy);
            unsafeAtomicAdd(g + 2 * (size_t)s.fps, vz);
        }
    }
}

template <int PREC>
__device__ __forceinline__ void b_edge_lj_gather(const Sys& s, int tile, double* tsh) {
    extern __shared__ double acc[];
    double* fi = tsh;                          // per-row sums
    int* hs = reinterpret_cast<int*>(tsh + 3 * kTile);  // the rows' half-list starts
    const int lane = threadIdx.x & (kWave - 1);
    const int cap = s.lds_cap;
    const int plane = lds_plane(cap);
    const int nseg = s.tile_nseg[tile];
    const bool staged = nseg >= 0;
    const int t0 = tile * kTile;
    const int nrow = min(kTile, s.n - t0);
    if (staged)
        for (int k = threadIdx.x; k < 3 * plane; k += kBlock) acc[k] = 0.0;
    if (threadIdx.x < 3 * kTile) fi[threadIdx.x] = 0.0;
    if (threadIdx.x <= nrow) hs[threadIdx.x] = s.hstart[t0 + threadIdx.x];
    __syncthreads();
    const int e0 = hs[0], e1 = hs[nrow];
    double* const P = s.fpl;  // force planes: component c of slot k at P[c * fps + k]
    const size_t fps = (size_t)s.fps;
    for (int base = e0; base < e1; base += kBlock) {
        const int e = base + threadIdx.x;
        const bool valid = e < e1;
        const int es = min(e, e1 - 1);
        int lo = 0, hi = nrow;  // hs[lo] <= es < hs[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (hs[mid] <= es) lo = mid;
            else hi = mid;
        }
        const int i = t0 + lo;
        const int ent = s.hj[es];
        const int j = min(entry_slot(ent), s.n - 1);
        const double4 xi = s.pos[i], xj = s.pos[j];
        const double dx = xj.x - xi.x + image(ent, 0, s.box);
        const double dy = xj.y - xi.y + image(ent, 1, s.box);
        const double dz = xj.z - xi.z + image(ent, 2, s.box);
        const double r2 = dx * dx + dy * dy + dz * dz;
        double fx = 0, fy = 0, fz = 0;
        if (valid && r2 < s.rc2) {
            if (PREC == 0) {
                double fr = lj_fr<double>(r2, s.l64, nullptr);
                fx = fr * dx;
                fy = fr * dy;
                fz = fr * dz;
            } else {
                float fr = lj_fr<float>((float)r2, s.l32, nullptr);
                fx = fr * (float)dx;
                fy = fr * (float)dy;
                fz = fr * (float)dz;
            }
        }
        const bool nz = (fx != 0.0) | (fy != 0.0) | (fz != 0.0);
        if (nz) {
            if (staged) {
                const int r = s.hr[es] & 0xffff;
                unsafeAtomicAdd(&acc[r], fx);
                unsafeAtomicAdd(&acc[plane + r], fy);
                unsafeAtomicAdd(&acc[2 * plane + r], fz);
            } else {
                unsafeAtomicAdd(P + j, fx);
                unsafeAtomicAdd(P + fps + j, fy);
                unsafeAtomicAdd(P + 2 * fps + j, fz);
            }
        }
        if (__any(nz)) {
            const int key = valid ? lo : kTile + lane;
            double sx = seg_sum(-fx, key, lane);
            double sy = seg_sum(-fy, key, lane);
            double sz = seg_sum(-fz, key, lane);
            int up = __shfl_up(key, 1);
            bool head = valid && (lane == 0 || up != key);
            if (head && ((sx != 0.0) | (sy != 0.0) | (sz != 0.0))) {
                unsafeAtomicAdd(&fi[3 * lo + 0], sx);
                unsafeAtomicAdd(&fi[3 * lo + 1], sy);
                unsafeAtomicAdd(&fi[3 * lo + 2], sz);
            }
        }
    }
    __syncthreads();
    if (staged) region_acc_flush(s, acc, plane, tile, P, fps, 1);
    edge_rows_flush(s, fi, t0, nrow);
}


template <int PREC>
__device__ __forceinline__ void lj_edge_pair(const Sys& s, double dx, double dy, double dz,
                                             double& fx, double& fy, double& fz) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    const bool in = r2 < s.rc2;
    if (PREC == 0) {
        const double inv = rcp_nr(r2);
        const double s2 = s.l64.sig2 * inv;
        const double s6 = s2 * s2 * s2;
        const double fr = s.l64.eps24 * inv * s6 * (2.0 * s6 - 1.0) * (in ? 1.0 : 0.0);
        fx = fr * dx;
        fy = fr * dy;
        fz = fr * dz;
    } else {
        const float r2f = (float)r2;
        const float inv = rcp_nr(r2f);
        const float s2 = s.l32.sig2 * inv;
        const float s6 = s2 * s2 * s2;
        const float fr = s.l32.eps24 * inv * s6 * (2.0f * s6 - 1.0f) * (in ? 1.0f : 0.0f);
        fx = fr * (float)dx;
        fy = fr * (float)dy;
        fz = fr * (float)dz;
    }
}

template <int PREC>
__device__ __forceinline__ void b_edge_lj_staged(const Sys& s, int tile, double* tsh) {
    extern __shared__ double lds3[];  // region positions, then the accumulator
    double* fi = tsh;                 // per-row sums
    double* xr = tsh + 3 * kTile;     // the tile's own positions
    const int cap = s.lds_cap;
    const int plane = lds_plane(cap);
    double* acc = lds3 + 3 * (cap + 1);
    const int t0 = tile * kTile;
    const int nrow = min(kTile, s.n - t0);
    const int e0 = s.hstart[t0], e1 = s.hstart[t0 + nrow];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int nchk = s.tile_nchunk[tile];
    RegionBatch rb;
    region_issue(s, s.pos, tile, nchk, wv, rb);
    // first block of packed entries: lane k takes entries a + 4k .. a + 4k + 3
    // (a = e0 rounded down to a multiple of four, so the load is aligned; the
    // allocation has four spare entries after the last)
    const int a0 = e0 & ~3;
    const int4* hw = reinterpret_cast<const int4*>(s.hr);
    int4 w = a0 + 4 * (int)threadIdx.x < e1 ? hw[(a0 >> 2) + threadIdx.x] : make_int4(0, 0, 0, 0);
    for (int k = threadIdx.x; k < 3 * plane; k += kBlock) acc[k] = 0.0;
    if (threadIdx.x < 3 * kTile) fi[threadIdx.x] = 0.0;
    if (threadIdx.x < nrow) {
        const double4 p = s.pos[t0 + threadIdx.x];
        xr[3 * threadIdx.x] = p.x;
        xr[3 * threadIdx.x + 1] = p.y;
        xr[3 * threadIdx.x + 2] = p.z;
    }
    region_store(s, lds3, rb);
    region_finish(s, s.pos, lds3, cap, tile, nchk, wv, rb);  // ends with the barrier
    for (int base = a0; base < e1; base += 4 * kBlock) {
        const int eb = base + 4 * (int)threadIdx.x;
        const int nxt = eb + 4 * kBlock;
        const int4 wn = nxt < e1 ? hw[(nxt >> 2)] : make_int4(0, 0, 0, 0);
        const int wd[4] = {w.x, w.y, w.z, w.w};
        int row[4], reg[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const bool ok = eb + u >= e0 && eb + u < e1;
            row[u] = ok ? (wd[u] >> 16) : -1;
            reg[u] = ok ? (wd[u] & 0xffff) : cap;  // the padding slot: no force
        }
        double gx[4], gy[4], gz[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int ri = max(row[u], 0);
            const double* pj = lds3 + 3 * reg[u];
            const double* pi = xr + 3 * ri;
            lj_edge_pair<PREC>(s, pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2], gx[u], gy[u], gz[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if ((gx[u] != 0.0) | (gy[u] != 0.0) | (gz[u] != 0.0)) {
                unsafeAtomicAdd(&acc[reg[u]], gx[u]);
                unsafeAtomicAdd(&acc[plane + reg[u]], gy[u]);
                unsafeAtomicAdd(&acc[2 * plane + reg[u]], gz[u]);
            }
        }
        // the row's share: the sum over each run of equal rows (rows ascend)
        double sx = 0, sy = 0, sz = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            sx -= gx[u];
            sy -= gy[u];
            sz -= gz[u];
            const bool last = u == 3 || row[u + 1] != row[u];
            if (last) {
                if (row[u] >= 0 && ((sx != 0.0) | (sy != 0.0) | (sz != 0.0))) {
                    unsafeAtomicAdd(&fi[3 * row[u]], sx);
                    unsafeAtomicAdd(&fi[3 * row[u] + 1], sy);
                    unsafeAtomicAdd(&fi[3 * row[u] + 2], sz);
                }
                sx = sy = sz = 0;
            }
        }
        w = wn;
    }
    __syncthreads();
    region_acc_flush(s, acc, plane, tile, s.fpl, (size_t)s.fps, 1);
    edge_rows_flush(s, fi, t0, nrow);
}

// STAGE: the launch's dynamic LDS holds the region copy as well
// (edge_lds_bytes), so staged tiles take b_edge_lj_staged.
template <int PREC, bool STAGE>
__device__ __forceinline__ void b_edge_lj_tile(const Sys& s, int tile, int nb) {
    // per-row sums, then the rows' positions (staged) or row starts (gather)
    __shared__ double tsh[6 * kTile];
    static_assert(sizeof(int) * (kTile + 1) <= sizeof(double) * 3 * kTile, "row starts fit");
    if (STAGE && s.tile_nseg[tile] >= 0) b_edge_lj_staged<PREC>(s, tile, tsh);
    else b_edge_lj_gather<PREC>(s, tile, tsh);
}

template <int PREC, bool STAGE>
__global__ __launch_bounds__(kBlock) void k_edge_lj_tile(Sys s) {
    b_edge_lj_tile<PREC, STAGE>(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// Patchy edge pass by tiles (patchy_edge_by_tile), one workgroup per tile of
// kTile rows, one lane per half-list entry (positions and orientations
// gathered from global memory).
// Each pair is evaluated once and zero results are skipped.  ACC, for a tile
// with a region: the partner's force and torque go into an LDS accumulator
// over the region (six planes), the row's share (combined over the lanes of
// the row by a segmented shuffle reduction) goes into the same accumulator at
// the row's own region index, so a particle that is both a row and a partner
// of the tile, or the partner of several rows, costs one global atomic per
// component at the end, when every non-zero accumulator is flushed (the
// region in runs of consecutive slots).  Other tiles add the partner's share
// with global atomics and the rows' shares through per-row LDS sums.  Forces
// and torques must be zero on entry.
constexpr int kPatchyAccCapMax = 2240;  // largest region accumulated in LDS
__host__ __device__ constexpr bool patchy_edge_accumulates(int cap) { return cap <= kPatchyAccCapMax; }
__host__ __device__ __forceinline__ size_t patchy_edge_lds_bytes(int cap) {
    return patchy_edge_accumulates(cap) ? 6 * sizeof(double) * (size_t)lds_plane(cap) : 0;
}

template <int PREC, bool ACC>
__device__ __forceinline__ void b_edge_patchy_tile(const Sys& s, int tile) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    extern __shared__ double acc[];
    __shared__ double fi[6 * kTile];  // per-row sums of tiles without a region
    __shared__ int hs[kTile + 1];     // the rows' half-list starts
    __shared__ int rreg[kTile];       // the rows' own region indices
    __shared__ int4 sg[kSegMax];
    const int lane = threadIdx.x & (kWave - 1);
    const int t0 = tile * kTile;
    const int nrow = min(kTile, s.n - t0);
    const int nseg = ACC ? s.tile_nseg[tile] : -1;
    const bool reg = nseg >= 0;
    const int plane = lds_plane(s.lds_cap);
    if (reg) {
        for (int k = threadIdx.x; k < 6 * plane; k += kBlock) acc[k] = 0.0;
        if (threadIdx.x < nseg) sg[threadIdx.x] = s.tile_seg[(size_t)tile * kSegMax + threadIdx.x];
    }
    for (int k = threadIdx.x; k < 6 * kTile; k += kBlock) fi[k] = 0.0;
    if (threadIdx.x <= nrow) hs[threadIdx.x] = s.hstart[t0 + threadIdx.x];
    __syncthreads();
    if (threadIdx.x < kTile)
        rreg[threadIdx.x] = reg && (int)threadIdx.x < nrow
                                ? tile_lds_base(sg, nseg, t0 + (int)threadIdx.x, kCodeHome)
                                : -1;
    __syncthreads();
    const int e0 = hs[0], e1 = hs[nrow];
    double* F = reinterpret_cast<double*>(s.frc);
    double* T = reinterpret_cast<double*>(s.trq);
    for (int base = e0; base < e1; base += kBlock) {
        const int e = base + threadIdx.x;
        const bool valid = e < e1;
        const int es = min(e, e1 - 1);
        int lo = 0, hi = nrow;  // hs[lo] <= es < hs[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (hs[mid] <= es) lo = mid;
            else hi = mid;
        }
        const int i = t0 + lo;
        const int ent = s.hj[es];
        const int j = min(entry_slot(ent), s.n - 1);
        const double4 xi = s.pos[i], xj = s.pos[j];
        const double dx = xj.x - xi.x + image(ent, 0, s.box);
        const double dy = xj.y - xi.y + image(ent, 1, s.box);
        const double dz = xj.z - xi.z + image(ent, 2, s.box);
        const double r2 = dx * dx + dy * dy + dz * dz;
        V3<double> fj = {0, 0, 0}, ti = {0, 0, 0}, tj = {0, 0, 0};
        if (valid && r2 < s.rc2) {
            V3<double> ui[4], uj[4];
            patch_dirs<double>(s.quat[i], ui, s.p64.model);
            patch_dirs<double>(s.quat[j], uj, s.p64.model);
            const V3<double> d = {dx, dy, dz};
            double v;
            patchy_pair<R>(d, r2, ui, uj, s, fj, ti, tj, v);
        }
        const bool fnz = (fj.x != 0.0) | (fj.y != 0.0) | (fj.z != 0.0);
        const bool tjnz = (tj.x != 0.0) | (tj.y != 0.0) | (tj.z != 0.0);
        const bool tinz = (ti.x != 0.0) | (ti.y != 0.0) | (ti.z != 0.0);
        // partner share: only non-zero results touch memory
        const int r = reg ? (int)(s.hr[es] & 0xffff) : kNoRegion;
        if (r != kNoRegion) {
            if (fnz) {
                unsafeAtomicAdd(&acc[r], fj.x);
                unsafeAtomicAdd(&acc[plane + r], fj.y);
                unsafeAtomicAdd(&acc[2 * plane + r], fj.z);
            }
            if (tjnz) {
                unsafeAtomicAdd(&acc[3 * plane + r], tj.x);
                unsafeAtomicAdd(&acc[4 * plane + r], tj.y);
                unsafeAtomicAdd(&acc[5 * plane + r], tj.z);
            }
        } else {
            if (fnz) {
                unsafeAtomicAdd(F + 4 * (size_t)j + 0, fj.x);
                unsafeAtomicAdd(F + 4 * (size_t)j + 1, fj.y);
                unsafeAtomicAdd(F + 4 * (size_t)j + 2, fj.z);
            }
            if (tjnz) {
                unsafeAtomicAdd(T + 4 * (size_t)j + 0, tj.x);
                unsafeAtomicAdd(T + 4 * (size_t)j + 1, tj.y);
                unsafeAtomicAdd(T + 4 * (size_t)j + 2, tj.z);
            }
        }
        // row share: the lanes of each row combined, one lane adds the sums
        if (__any(fnz | tinz)) {
            const int key = valid ? lo : kTile + lane;
            const double sx = seg_sum(-fj.x, key, lane);
            const double sy = seg_sum(-fj.y, key, lane);
            const double sz = seg_sum(-fj.z, key, lane);
            const double ux = seg_sum(ti.x, key, lane);
            const double uy = seg_sum(ti.y, key, lane);
            const double uz = seg_sum(ti.z, key, lane);
            const int up = __shfl_up(key, 1);
            const bool head = valid && (lane == 0 || up != key);
            if (head) {
                const int rr = rreg[lo];
                double* a = rr >= 0 ? acc + rr : fi + 6 * lo;
                const int st = rr >= 0 ? plane : 1;
                if ((sx != 0.0) | (sy != 0.0) | (sz != 0.0)) {
                    unsafeAtomicAdd(a, sx);
                    unsafeAtomicAdd(a + st, sy);
                    unsafeAtomicAdd(a + 2 * st, sz);
                }
                if ((ux != 0.0) | (uy != 0.0) | (uz != 0.0)) {
                    unsafeAtomicAdd(a + 3 * st, ux);
                    unsafeAtomicAdd(a + 4 * st, uy);
                    unsafeAtomicAdd(a + 5 * st, uz);
                }
            }
        }
    }
    __syncthreads();
    if (reg) {
        region_acc_flush(s, acc, plane, tile, F);
        region_acc_flush(s, acc + 3 * plane, plane, tile, T);
    }
    if (threadIdx.x < nrow) {
        const double* a = fi + 6 * threadIdx.x;
        double* g = F + 4 * (size_t)(t0 + threadIdx.x);
        double* h = T + 4 * (size_t)(t0 + threadIdx.x);
        if ((a[0] != 0.0) | (a[1] != 0.0) | (a[2] != 0.0)) {
            unsafeAtomicAdd(g + 0, a[0]);
            unsafeAtomicAdd(g + 1, a[1]);
            unsafeAtomicAdd(g + 2, a[2]);
        }
        if ((a[3] != 0.0) | (a[4] != 0.0) | (a[5] != 0.0)) {
            unsafeAtomicAdd(h + 0, a[3]);
            unsafeAtomicAdd(h + 1, a[4]);
            unsafeAtomicAdd(h + 2, a[5]);
        }
    }
}

template <int PREC, bool ACC>
__global__ __launch_bounds__(kBlock) void k_edge_patchy_tile(Sys s) {
    b_edge_patchy_tile<PREC, ACC>(s, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Vertex decomposition with Newton's third law (LJ).  The TPP lanes of
// particle i walk its half list (partners j > i), evaluate each pair once,
// keep -F_ij for i in registers and add +F_ij to j atomically, skipping exact
// zeros.  REP: the partner share goes into one of nrep replicated force
// arrays (chosen per wavefront), i's own sum is stored straight into F (its
// only writer), and a combining pass adds the replicas to F and clears them.
// !REP: the partner share of a staged tile goes into an LDS accumulator over
// the tile's region, added once per workgroup (region_acc_flush); i's own sum
// and unstaged partners are added atomically.  These adds go to the force
// planes (as in the edge pass), which must be zero on entry.
// ---------------------------------------------------------------------------
template <int PREC, bool REP>
__device__ __forceinline__ void b_newton_lj(const Sys& s, int tile, int nb) {
    extern __shared__ double acc[];
    constexpr int TPP = kTileTpp;
    const int cap = s.lds_cap;
    const int plane = lds_plane(cap);
    const bool staged = !REP && s.tile_nseg[tile] >= 0;
    if (!REP) {
        if (staged)
            for (int k = threadIdx.x; k < 3 * plane; k += kBlock) acc[k] = 0.0;
        __syncthreads();
    }
    const int i = tile * kTile + threadIdx.x / TPP;
    const int q = threadIdx.x % TPP;
    const bool act = i < s.n;
    const int ii = act ? i : s.n - 1;
    const int e0 = act ? s.hstart[ii] : 0;
    const int e1 = act ? s.hstart[ii + 1] : 0;
    const double4 xi = s.pos[ii];
    double* Rp = nullptr;
    if (REP) {
        const long long wave = (long long)tile * (kBlock / kWave) + threadIdx.x / kWave;
        Rp = reinterpret_cast<double*>(s.rep + (size_t)(wave % s.nrep) * s.n);
    }
    double fx = 0, fy = 0, fz = 0;
    for (int e = e0 + q; e < e1; e += TPP) {
        const int ent = s.hj[e];
        const int j = min(entry_slot(ent), s.n - 1);
        const double4 xj = s.pos[j];
        const double dx = xj.x - xi.x + image(ent, 0, s.box);
        const double dy = xj.y - xi.y + image(ent, 1, s.box);
        const double dz = xj.z - xi.z + image(ent, 2, s.box);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < s.rc2) {
            double gx, gy, gz;  // force on j
            if (PREC == 0) {
                double fr = lj_fr<double>(r2, s.l64, nullptr);
                gx = fr * dx;
                gy = fr * dy;
                gz = fr * dz;
            } else {
                float fr = lj_fr<float>((float)r2, s.l32, nullptr);
                gx = fr * (float)dx;
                gy = fr * (float)dy;
                gz = fr * (float)dz;
            }
            fx -= gx;
            fy -= gy;
            fz -= gz;
            if ((gx != 0.0) | (gy != 0.0) | (gz != 0.0)) {
                if (staged) {
                    const int r = s.hr[e] & 0xffff;
                    unsafeAtomicAdd(&acc[r], gx);
                    unsafeAtomicAdd(&acc[plane + r], gy);
                    unsafeAtomicAdd(&acc[2 * plane + r], gz);
                } else if (REP) {
                    double* g = Rp + 4 * (size_t)j;
                    unsafeAtomicAdd(g + 0, gx);
                    unsafeAtomicAdd(g + 1, gy);
                    unsafeAtomicAdd(g + 2, gz);
                } else {
                    unsafeAtomicAdd(s.fpl + j, gx);
                    unsafeAtomicAdd(s.fpl + s.fps + j, gy);
                    unsafeAtomicAdd(s.fpl + 2 * (size_t)s.fps + j, gz);
                }
            }
        }
    }
#pragma unroll
    for (int off = TPP / 2; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
    }
    if (act && q == 0) {
        if (REP) {
            s.frc[i] = make_double4(fx, fy, fz, 0.0);
        } else if ((fx != 0.0) | (fy != 0.0) | (fz != 0.0)) {
            unsafeAtomicAdd(s.fpl + i, fx);
            unsafeAtomicAdd(s.fpl + s.fps + i, fy);
            unsafeAtomicAdd(s.fpl + 2 * (size_t)s.fps + i, fz);
        }
    }
    if (!REP) {
        __syncthreads();
        if (staged) region_acc_flush(s, acc, plane, tile, s.fpl, (size_t)s.fps, 1);
    }
}

template <int PREC, bool REP>
__global__ __launch_bounds__(kBlock) void k_newton_lj(Sys s) {
    b_newton_lj<PREC, REP>(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// Newton's-third-law vertex pass for patchy particles (the paper's Discussion
// section: where it pays, it does so for the models with few, expensive
// interactions).  TPP lanes per particle (patchy_vertex_tpp) walk its half
// list; each pair is evaluated once, -F_ij and tau_i stay in registers, +F_ij
// and tau_j go to the partner atomically, each skipped when exactly zero.
// REP: into one of nrep replicated force and torque arrays (chosen per
// wavefront), i's own sums stored straight into F and tau (their only
// writer), then k_newton_combine; !REP: device-scope atomics into F and tau,
// which must be zero on entry (the patchy passes stage no region in LDS).
template <int PREC, bool REP, int TPP>
__device__ __forceinline__ void b_newton_patchy(const Sys& s, int bid, int nb) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    const int i = bid * (kBlock / TPP) + (int)threadIdx.x / TPP;
    const int q = (int)threadIdx.x % TPP;
    const bool act = i < s.n;
    const int ii = act ? i : s.n - 1;
    const int e0 = act ? s.hstart[ii] : 0;
    const int e1 = act ? s.hstart[ii + 1] : 0;
    const double4 xi = s.pos[ii];
    V3<double> ui[4];
    patch_dirs<double>(s.quat[ii], ui, s.p64.model);
    double* F = reinterpret_cast<double*>(s.frc);
    double* T = reinterpret_cast<double*>(s.trq);
    if (REP) {
        const long long wave = ((long long)bid * kBlock + threadIdx.x) / kWave;
        const size_t r = (size_t)(wave % s.nrep);
        F = reinterpret_cast<double*>(s.rep + r * s.n);
        T = reinterpret_cast<double*>(s.rep + (s.nrep + r) * (size_t)s.n);
    }
    Acc3<PREC> f, tq;
    for (int e = e0 + q; e < e1; e += TPP) {
        const int ent = s.hj[e];
        const int j = min(entry_slot(ent), s.n - 1);
        const double4 xj = s.pos[j];
        const double dx = xj.x - xi.x + image(ent, 0, s.box);
        const double dy = xj.y - xi.y + image(ent, 1, s.box);
        const double dz = xj.z - xi.z + image(ent, 2, s.box);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < s.rc2)) continue;
        V3<double> uj[4];
        patch_dirs<double>(s.quat[j], uj, s.p64.model);
        const V3<double> d = {dx, dy, dz};
        V3<double> fj, ti, tj;
        double v;
        patchy_pair<R>(d, r2, ui, uj, s, fj, ti, tj, v);
        f.add(-fj.x, -fj.y, -fj.z);
        tq.add(ti.x, ti.y, ti.z);
        if ((fj.x != 0.0) | (fj.y != 0.0) | (fj.z != 0.0)) {
            double* g = F + 4 * (size_t)j;
            unsafeAtomicAdd(g + 0, fj.x);
            unsafeAtomicAdd(g + 1, fj.y);
            unsafeAtomicAdd(g + 2, fj.z);
        }
        if ((tj.x != 0.0) | (tj.y != 0.0) | (tj.z != 0.0)) {
            double* g = T + 4 * (size_t)j;
            unsafeAtomicAdd(g + 0, tj.x);
            unsafeAtomicAdd(g + 1, tj.y);
            unsafeAtomicAdd(g + 2, tj.z);
        }
    }
    double fx = f.gx(), fy = f.gy(), fz = f.gz();
    double tx = tq.gx(), ty = tq.gy(), tz = tq.gz();
#pragma unroll
    for (int off = 1; off < TPP; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
        tx += __shfl_xor(tx, off);
        ty += __shfl_xor(ty, off);
        tz += __shfl_xor(tz, off);
    }
    if (!act || q != 0) return;
    if (REP) {
        s.frc[i] = make_double4(fx, fy, fz, 0.0);
        s.trq[i] = make_double4(tx, ty, tz, 0.0);
        return;
    }
    double* Fi = reinterpret_cast<double*>(s.frc) + 4 * (size_t)i;
    double* Ti = reinterpret_cast<double*>(s.trq) + 4 * (size_t)i;
    if ((fx != 0.0) | (fy != 0.0) | (fz != 0.0)) {
        unsafeAtomicAdd(Fi + 0, fx);
        unsafeAtomicAdd(Fi + 1, fy);
        unsafeAtomicAdd(Fi + 2, fz);
    }
    if ((tx != 0.0) | (ty != 0.0) | (tz != 0.0)) {
        unsafeAtomicAdd(Ti + 0, tx);
        unsafeAtomicAdd(Ti + 1, ty);
        unsafeAtomicAdd(Ti + 2, tz);
    }
}

template <int PREC, bool REP, int TPP>
__global__ __launch_bounds__(kBlock) void k_newton_patchy(Sys s) {
    b_newton_patchy<PREC, REP, TPP>(s, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// Closing pass of the replicated Newton mode: F (and tau) += sum of the
// replicas, which are cleared for the next pass; optionally the closing half
// kick (and the angular one).  Patchy replicas: nrep force arrays, then nrep
// torque arrays.
template <bool KICK>
__global__ __launch_bounds__(kBlock) void k_newton_combine(Sys s) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (KICK && blockIdx.x == 0 && threadIdx.x == 0) s.ctrl->rebuild = 0;
    if (i >= s.n) return;
    double4 f = s.frc[i];
    for (int r = 0; r < s.nrep; r++) {
        double4* p = s.rep + (size_t)r * s.n + i;
        const double4 v = *p;
        f.x += v.x;
        f.y += v.y;
        f.z += v.z;
        *p = make_double4(0.0, 0.0, 0.0, 0.0);
    }
    s.frc[i] = f;
    double4 tq = make_double4(0.0, 0.0, 0.0, 0.0);
    if (s.pot == 1) {
        tq = s.trq[i];
        for (int r = 0; r < s.nrep; r++) {
            double4* p = s.rep + (size_t)(s.nrep + r) * s.n + i;
            const double4 v = *p;
            tq.x += v.x;
            tq.y += v.y;
            tq.z += v.z;
            *p = make_double4(0.0, 0.0, 0.0, 0.0);
        }
        s.trq[i] = tq;
    }
    if (!isfinite(f.x + f.y + f.z + tq.x + tq.y + tq.z)) atomicOr(&s.ctrl->nonfinite, 1);
    if (KICK) {
        double4 v = s.vel[i];
        v.x += s.hdt * f.x * s.inv_mass;
        v.y += s.hdt * f.y * s.inv_mass;
        v.z += s.hdt * f.z * s.inv_mass;
        s.vel[i] = v;
        if (s.pot == 1) {
            double4 L = s.angm[i];
            L.x += s.hdt * tq.x;
            L.y += s.hdt * tq.y;
            L.z += s.hdt * tq.z;
            s.angm[i] = L;
        }
    }
}

// ---------------------------------------------------------------------------
// Velocity Verlet (FP64).  kick_drift: v += dt/2 F/m, x += dt v, wrap into
// [0, L); patchy also L += dt/2 tau and a free rotation of q by |L|/I dt
// about L.  Flags a rebuild if any particle moved more than skin/2 since the
// last build.  Optionally zeroes F (and tau) for the edge pass.
// ---------------------------------------------------------------------------

template <int POT, bool ZERO>
__device__ __forceinline__ void b_kick_drift(const Sys& s, int bid, int nb) {
    int i = bid * kBlock + threadIdx.x;
    if (i >= s.n) return;
    double4 f = s.frc[i];
    double4 v = s.vel[i];
    double4 x = s.pos[i];
    v.x += s.hdt * f.x * s.inv_mass;
    v.y += s.hdt * f.y * s.inv_mass;
    v.z += s.hdt * f.z * s.inv_mass;
    x.x += s.dt * v.x;  // unwrapped until the next list build
    x.y += s.dt * v.y;
    x.z += s.dt * v.z;
    s.vel[i] = v;
    s.pos[i] = x;
    if (POT == 1) {
        double4 tq = s.trq[i];
        double4 L = s.angm[i];
        L.x += s.hdt * tq.x;
        L.y += s.hdt * tq.y;
        L.z += s.hdt * tq.z;
        s.angm[i] = L;
        double Ln = sqrt(L.x * L.x + L.y * L.y + L.z * L.z);
        if (Ln > 0) {
            double th = Ln * s.inv_inertia * s.dt;
            double sh, ch;
            sincos(0.5 * th, &sh, &ch);
            double ax = sh * L.x / Ln, ay = sh * L.y / Ln, az = sh * L.z / Ln;
            double4 q = s.quat[i];  // (w, x, y, z) in (x, y, z, w) slots
            double nw = ch * q.x - ax * q.y - ay * q.z - az * q.w;
            double nx = ch * q.y + ax * q.x + ay * q.w - az * q.z;
            double ny = ch * q.z - ax * q.w + ay * q.x + az * q.y;
            double nz = ch * q.w + ax * q.z - ay * q.y + az * q.x;
            double inv = 1.0 / sqrt(nw * nw + nx * nx + ny * ny + nz * nz);
            s.quat[i] = make_double4(nw * inv, nx * inv, ny * inv, nz * inv);
        }
        if (ZERO) s.trq[i] = make_double4(0, 0, 0, 0);
    }
    if (ZERO) {
        s.frc[i] = make_double4(0, 0, 0, 0);
        if (POT == 0) {  // the LJ edge pass adds into the force planes
            s.fpl[i] = 0.0;
            s.fpl[s.fps + i] = 0.0;
            s.fpl[2 * (size_t)s.fps + i] = 0.0;
        }
    }
    double4 xb = s.xbuild[i];
    double ddx = x.x - xb.x;
    double ddy = x.y - xb.y;
    double ddz = x.z - xb.z;
    if (ddx * ddx + ddy * ddy + ddz * ddz > s.disp2) s.ctrl->rebuild = 1;
}

template <int POT, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_kick_drift(Sys s) { b_kick_drift<POT, ZERO>(s, blockIdx.x, gridDim.x); }

// PLANES (LJ edge pass): the forces come from the force planes and are
// stored into the force records on the way.
template <int POT, bool PLANES = false>
__device__ __forceinline__ void b_kick(const Sys& s, int bid, int nb) {
    int i = bid * kBlock + threadIdx.x;
    if (bid == 0 && threadIdx.x == 0) s.ctrl->rebuild = 0;
    if (i >= s.n) return;
    double4 f;
    if (PLANES) {
        f = make_double4(s.fpl[i], s.fpl[s.fps + i], s.fpl[2 * (size_t)s.fps + i], 0.0);
        s.frc[i] = f;
    } else {
        f = s.frc[i];
    }
    double4 v = s.vel[i];
    v.x += s.hdt * f.x * s.inv_mass;
    v.y += s.hdt * f.y * s.inv_mass;
    v.z += s.hdt * f.z * s.inv_mass;
    s.vel[i] = v;
    double chk = f.x + f.y + f.z;
    if (POT == 1) {
        double4 tq = s.trq[i];
        double4 L = s.angm[i];
        L.x += s.hdt * tq.x;
        L.y += s.hdt * tq.y;
        L.z += s.hdt * tq.z;
        s.angm[i] = L;
        chk += tq.x + tq.y + tq.z;
    }
    if (!isfinite(chk)) atomicOr(&s.ctrl->nonfinite, 1);
}

template <int POT, bool PLANES = false>
__global__ __launch_bounds__(kBlock) void k_kick(Sys s) { b_kick<POT, PLANES>(s, blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(kBlock) void k_zero_forces(Sys s) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    s.frc[i] = make_double4(0, 0, 0, 0);
    if (s.pot == 1) {
        s.trq[i] = make_double4(0, 0, 0, 0);
    } else {
        s.fpl[i] = 0.0;
        s.fpl[s.fps + i] = 0.0;
        s.fpl[2 * (size_t)s.fps + i] = 0.0;
    }
}

// Force records from the force planes (LJ edge pass without a kick).
__global__ __launch_bounds__(kBlock) void k_forces_from_planes(Sys s) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const double fx = s.fpl[i], fy = s.fpl[s.fps + i], fz = s.fpl[2 * (size_t)s.fps + i];
    s.frc[i] = make_double4(fx, fy, fz, 0.0);
    if (!isfinite(fx + fy + fz)) atomicOr(&s.ctrl->nonfinite, 1);
}

// Clears the rebuild flag after a stand-alone edge pass (the vertex kernel
// clears it itself).
__global__ void k_clear_rebuild(Ctrl* c) { c->rebuild = 0; }

// ---------------------------------------------------------------------------
// Energies: per-particle terms (vertex-style walk of the full list), then a
// fixed-shape FP64 tree reduction: kRedBlocks partial sums over fixed index
// ranges, then one block sums the partials.  Deterministic for a given order.
// ---------------------------------------------------------------------------

template <int POT>
__global__ __launch_bounds__(kBlock) void k_kinetic(Sys s) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    double4 v = s.vel[i];
    double k = 0.5 * (v.x * v.x + v.y * v.y + v.z * v.z) / s.inv_mass;
    if (POT == 1) {
        double4 L = s.angm[i];
        k += 0.5 * (L.x * L.x + L.y * L.y + L.z * L.z) * s.inv_inertia;
    }
    s.kpart[i] = k;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x / kWave); w++) t += sh[w];
    return t;
}

__global__ __launch_bounds__(kBlock) void k_reduce_partial(Sys s) {
    __shared__ double sh[kBlock / kWave];
    int per = (s.n + kRedBlocks - 1) / kRedBlocks;
    int b = blockIdx.x * per;
    int e = min(b + per, s.n);
    const double* src[3] = {s.kpart, s.epart, s.wpart};
    for (int q = 0; q < 3; q++) {
        double v = 0;
        for (int k = b + threadIdx.x; k < e; k += kBlock) v += src[q][k];
        double t = block_sum(v, sh);
        if (threadIdx.x == 0) s.red[q * kRedBlocks + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kRedBlocks) void k_reduce_final(Sys s) {
    __shared__ double sh[kRedBlocks / kWave];
    for (int q = 0; q < 3; q++) {
        double v = s.red[q * kRedBlocks + threadIdx.x];
        double t = block_sum(v, sh);
        if (threadIdx.x == 0) s.red[3 * kRedBlocks + q] = t;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline dim3 grid_n(int n) { return dim3((n + kBlock - 1) / kBlock); }

hipError_t launch_set_rebuild(const Sys& s, hipStream_t st) {
    hipLaunchKernelGGL(k_set_rebuild, dim3(1), dim3(1), 0, st, s.ctrl);
    return hipGetLastError();
}

hipError_t launch_clear_ctrl(const Sys& s, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_ctrl, dim3(1), dim3(kBlock), 0, st, s.ctrl, s.sync);
    return hipGetLastError();
}

hipError_t launch_rebuild(const Sys& s, hipStream_t st, bool cells, bool lists) {
    // cells: bin (+ scan by the last workgroup), scatter, sort + reorder beside
    // the tile regions; lists: build (+ half-list offsets by the last
    // workgroup); the half list itself is filled on demand (launch_half_fill)
    if (cells) {
        hipLaunchKernelGGL(k_cell_bin, grid_n(s.n), dim3(kBlock), 0, st, s);
        hipLaunchKernelGGL(k_cell_scatter, grid_n(s.n), dim3(kBlock), 0, st, s);
        hipLaunchKernelGGL(k_sort_tiles, dim3((unsigned)class_blocks(s, kClsSortTiles)),
                           dim3(kBlock), 0, st, s);
    }
    if (lists) hipLaunchKernelGGL(k_build, dim3(s.nblk), dim3(kBlock), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_half_fill(const Sys& s, hipStream_t st) {
    size_t sh_map = sizeof(int) * (size_t)(s.lds_cap + 8);
    hipLaunchKernelGGL(k_half_fill, dim3(s.ntiles), dim3(kBlock), sh_map, st, s);
    if (s.estore) hipLaunchKernelGGL(k_col_fill, dim3(s.ntiles), dim3(kBlock), sh_map, st, s);
    return hipGetLastError();
}

void set_potential(Sys& s, double eps, double sigma, double rc, double eps_p, double w,
                   double delta, double rpc, int patch_model) {
    double s2 = sigma * sigma / (rc * rc);
    double s6 = s2 * s2 * s2;
    double vs = 4.0 * eps * (s6 * s6 - s6);
    const double sig6 = sigma * sigma * sigma * sigma * sigma * sigma;
    s.l64 = {sigma * sigma, 4.0 * eps, 24.0 * eps, rc * rc, vs, 48.0 * eps * sig6 * sig6,
             24.0 * eps * sig6};
    s.l32 = {(float)(sigma * sigma), (float)(4.0 * eps), (float)(24.0 * eps), (float)(rc * rc),
             (float)vs, (float)(48.0 * eps * sig6 * sig6), (float)(24.0 * eps * sig6)};
    double wca2 = cbrt(2.0) * sigma * sigma;
    double rpc2 = rpc > 0 ? rpc * rpc : 0.0;
    s.p64 = {sigma * sigma, 4.0 * eps, 24.0 * eps, eps, wca2, eps_p, 1.0 / (w * w), delta, rpc2,
             patch_model};
    s.p32 = {(float)(sigma * sigma), (float)(4.0 * eps), (float)(24.0 * eps), (float)eps,
             (float)wca2, (float)eps_p, (float)(1.0 / (w * w)), (float)delta, (float)rpc2,
             patch_model};
}

template <int PREC>
static void vertex_dispatch(const Sys& s, bool kick, bool energy, hipStream_t st,
                            bool drift = false) {
    dim3 b(kBlock);
    if (s.pot == 0) {
        constexpr int T = kTileTpp;
        dim3 gl((unsigned)s.ntiles);
        size_t sh = lds_region_bytes(s.lds_cap);
        if (kick && drift)
            hipLaunchKernelGGL((k_vertex_lj<PREC, T, true, false, true>), gl, b, sh, st, s);
        else if (kick)
            hipLaunchKernelGGL((k_vertex_lj<PREC, T, true, false>), gl, b, sh, st, s);
        else if (energy)
            hipLaunchKernelGGL((k_vertex_lj<PREC, T, false, true>), gl, b, sh, st, s);
        else
            hipLaunchKernelGGL((k_vertex_lj<PREC, T, false, false>), gl, b, sh, st, s);
    } else if (patchy_vertex_tpp(s) > 1) {
        constexpr int T = kTileTpp;
        dim3 gt((unsigned)s.ntiles);  // one tile of particles per workgroup
        if (kick)
            hipLaunchKernelGGL((k_vertex_patchy<PREC, true, false, T>), gt, b, 0, st, s);
        else if (energy)
            hipLaunchKernelGGL((k_vertex_patchy<PREC, false, true, T>), gt, b, 0, st, s);
        else
            hipLaunchKernelGGL((k_vertex_patchy<PREC, false, false, T>), gt, b, 0, st, s);
    } else {
        dim3 g((unsigned)s.nblk);  // one lane per particle
        if (kick)
            hipLaunchKernelGGL((k_vertex_patchy<PREC, true, false, 1>), g, b, 0, st, s);
        else if (energy)
            hipLaunchKernelGGL((k_vertex_patchy<PREC, false, true, 1>), g, b, 0, st, s);
        else
            hipLaunchKernelGGL((k_vertex_patchy<PREC, false, false, 1>), g, b, 0, st, s);
    }
}

template <int PREC>
static void edge_dispatch(const Sys& s, int grid, hipStream_t st) {
    dim3 g(grid), b(kBlock);
    if (s.pot == 0) {
        const size_t sh = edge_lds_bytes(s.lds_cap);
        if (edge_stages_positions(s.lds_cap))
            hipLaunchKernelGGL((k_edge_lj_tile<PREC, true>), dim3((unsigned)s.ntiles), b, sh, st, s);
        else
            hipLaunchKernelGGL((k_edge_lj_tile<PREC, false>), dim3((unsigned)s.ntiles), b, sh, st, s);
    } else if (!patchy_edge_by_tile(s)) {
        hipLaunchKernelGGL((k_edge<1, PREC>), g, b, 0, st, s);
    } else if (patchy_edge_accumulates(s.lds_cap)) {
        hipLaunchKernelGGL((k_edge_patchy_tile<PREC, true>), dim3((unsigned)s.ntiles), b,
                           patchy_edge_lds_bytes(s.lds_cap), st, s);
    } else {
        hipLaunchKernelGGL((k_edge_patchy_tile<PREC, false>), dim3((unsigned)s.ntiles), b, 0, st, s);
    }
}

template <int PREC>
static void newton_dispatch(const Sys& s, hipStream_t st) {
    dim3 g((unsigned)s.ntiles), b(kBlock);
    if (s.pot == 1) {
        const bool lanes = patchy_vertex_tpp(s) > 1;
        const dim3 gp((unsigned)(lanes ? s.ntiles : s.nblk));
        if (s.nrep > 0) {
            if (lanes) hipLaunchKernelGGL((k_newton_patchy<PREC, true, kTileTpp>), gp, b, 0, st, s);
            else hipLaunchKernelGGL((k_newton_patchy<PREC, true, 1>), gp, b, 0, st, s);
        } else {
            if (lanes) hipLaunchKernelGGL((k_newton_patchy<PREC, false, kTileTpp>), gp, b, 0, st, s);
            else hipLaunchKernelGGL((k_newton_patchy<PREC, false, 1>), gp, b, 0, st, s);
        }
        return;
    }
    if (s.nrep > 0) {
        hipLaunchKernelGGL((k_newton_lj<PREC, true>), g, b, 0, st, s);
    } else {
        size_t sh = lds_acc_bytes(s.lds_cap);
        hipLaunchKernelGGL((k_newton_lj<PREC, false>), g, b, sh, st, s);
    }
}

hipError_t launch_forces(const Sys& s, int mode, int prec, bool kick, hipStream_t st, int edge_grid,
                         hipEvent_t mid) {
    // closing kick of the passes without a fused one, after the `mid` event
    auto closing_kick = [&](bool newton_combine) {
        if (mid) (void)hipEventRecord(mid, st);  // an error surfaces below
        if (newton_combine) hipLaunchKernelGGL(k_newton_combine<true>, grid_n(s.n), dim3(kBlock), 0, st, s);
        else if (s.pot == 0) hipLaunchKernelGGL(k_kick<0>, grid_n(s.n), dim3(kBlock), 0, st, s);
        else hipLaunchKernelGGL(k_kick<1>, grid_n(s.n), dim3(kBlock), 0, st, s);
    };
    if (mode == 0) {
        if (prec == 0) vertex_dispatch<0>(s, kick, false, st);
        else if (prec == 1) vertex_dispatch<1>(s, kick, false, st);
        else vertex_dispatch<2>(s, kick, false, st);
        if (kick && mid) (void)hipEventRecord(mid, st);
    } else if (mode == 2) {  // Newton; with atomics into F (and tau) it must start at zero
        (void)launch_half_fill(s, st);  // launch errors surface in hipGetLastError below
        if (s.nrep == 0 && !kick) hipLaunchKernelGGL(k_zero_forces, grid_n(s.n), dim3(kBlock), 0, st, s);
        if (prec == 0) newton_dispatch<0>(s, st);
        else newton_dispatch<1>(s, st);  // FP32 pair maths, FP64 sums
        const bool planes = s.pot == 0 && s.nrep == 0;  // LJ with LDS accumulation
        if (kick && planes) {
            if (mid) (void)hipEventRecord(mid, st);
            hipLaunchKernelGGL((k_kick<0, true>), grid_n(s.n), dim3(kBlock), 0, st, s);
        } else if (kick) {
            closing_kick(s.nrep > 0);
        } else if (s.nrep > 0) {
            hipLaunchKernelGGL(k_newton_combine<false>, grid_n(s.n), dim3(kBlock), 0, st, s);
        } else if (planes) {
            hipLaunchKernelGGL(k_forces_from_planes, grid_n(s.n), dim3(kBlock), 0, st, s);
        }
        if (!kick) hipLaunchKernelGGL(k_clear_rebuild, dim3(1), dim3(1), 0, st, s.ctrl);
    } else if (mode == 3) {  // deterministic edge: per-edge results, then a gather
        if (!s.estore) return hipErrorInvalidValue;
        (void)launch_half_fill(s, st);  // launch errors surface in hipGetLastError below
        dim3 g((unsigned)edge_grid), b(kBlock);
        if (s.pot == 0) {
            if (prec == 0) hipLaunchKernelGGL((k_edge<0, 0, true>), g, b, 0, st, s);
            else hipLaunchKernelGGL((k_edge<0, 1, true>), g, b, 0, st, s);
            hipLaunchKernelGGL(k_edge_gather<0>, dim3((unsigned)s.ntiles), b, 0, st, s);
        } else {
            if (prec == 0) hipLaunchKernelGGL((k_edge<1, 0, true>), g, b, 0, st, s);
            else hipLaunchKernelGGL((k_edge<1, 1, true>), g, b, 0, st, s);
            hipLaunchKernelGGL(k_edge_gather<1>, dim3((unsigned)s.ntiles), b, 0, st, s);
        }
        if (kick) closing_kick(false);
        else hipLaunchKernelGGL(k_clear_rebuild, dim3(1), dim3(1), 0, st, s.ctrl);
    } else {
        (void)launch_half_fill(s, st);  // launch errors surface in hipGetLastError below
        if (!kick) hipLaunchKernelGGL(k_zero_forces, grid_n(s.n), dim3(kBlock), 0, st, s);
        if (prec == 0) edge_dispatch<0>(s, edge_grid, st);
        else edge_dispatch<1>(s, edge_grid, st);  // FP32 pair maths, FP64 atomics
        if (kick && s.pot == 0) {  // LJ: the forces are in the planes
            if (mid) (void)hipEventRecord(mid, st);
            hipLaunchKernelGGL((k_kick<0, true>), grid_n(s.n), dim3(kBlock), 0, st, s);
        } else if (kick) {
            closing_kick(false);
        } else {
            if (s.pot == 0) hipLaunchKernelGGL(k_forces_from_planes, grid_n(s.n), dim3(kBlock), 0, st, s);
            hipLaunchKernelGGL(k_clear_rebuild, dim3(1), dim3(1), 0, st, s.ctrl);
        }
    }
    return hipGetLastError();
}

hipError_t launch_vertex_kick_drift(const Sys& s, int prec, hipStream_t st) {
    if (s.pot != 0) return hipErrorInvalidValue;
    if (prec == 0) vertex_dispatch<0>(s, true, false, st, true);
    else if (prec == 1) vertex_dispatch<1>(s, true, false, st, true);
    else vertex_dispatch<2>(s, true, false, st, true);
    return hipGetLastError();
}

hipError_t launch_clear_rebuild(const Sys& s, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_rebuild, dim3(1), dim3(1), 0, st, s.ctrl);
    return hipGetLastError();
}

hipError_t launch_kick_drift(const Sys& s, bool zero_forces, hipStream_t st) {
    if (s.pot == 0) {
        if (zero_forces) hipLaunchKernelGGL((k_kick_drift<0, true>), grid_n(s.n), dim3(kBlock), 0, st, s);
        else hipLaunchKernelGGL((k_kick_drift<0, false>), grid_n(s.n), dim3(kBlock), 0, st, s);
    } else {
        if (zero_forces) hipLaunchKernelGGL((k_kick_drift<1, true>), grid_n(s.n), dim3(kBlock), 0, st, s);
        else hipLaunchKernelGGL((k_kick_drift<1, false>), grid_n(s.n), dim3(kBlock), 0, st, s);
    }
    return hipGetLastError();
}

hipError_t launch_kick(const Sys& s, hipStream_t st) {
    if (s.pot == 0) hipLaunchKernelGGL(k_kick<0>, grid_n(s.n), dim3(kBlock), 0, st, s);
    else hipLaunchKernelGGL(k_kick<1>, grid_n(s.n), dim3(kBlock), 0, st, s);
    return hipGetLastError();
}

// Energy pass: per-particle potential energy and virial (vertex walk in the
// configured precision, forces rewritten identically), kinetic terms, and the
// fixed-order reduction into s.red[3 * kRedBlocks + {0,1,2}].
// ---------------------------------------------------------------------------
// NVT thermostat: each particle's momenta are redrawn from the
// Maxwell-Boltzmann distribution with probability prob (Methods section, the
// Brownian scheme it cites).  Random numbers come from Philox4x64-10 (Salmon,
// Moraes, Dror and Shaw, SC 2011) keyed by (seed, 0), counter (particle id,
// call counter, block, 0), so a particle's draws follow it through every
// re-sort of the slots.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t h0 = __umul64hi(M0, x[0]), l0 = M0 * x[0];
        const uint64_t h1 = __umul64hi(M1, x[2]), l1 = M1 * x[2];
        const uint64_t y0 = h1 ^ x[1] ^ k0, y2 = h0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = l1;
        x[2] = y2;
        x[3] = l0;
    }
}

// (0, 1) from the top 53 bits
__device__ __forceinline__ double unit53(uint64_t r) {
    return ((double)(r >> 11) + 0.5) * 0x1.0p-53;
}

// two standard normals (Box-Muller) from two words
__device__ __forceinline__ void box_muller(uint64_t a, uint64_t b, double& g0, double& g1) {
    const double rad = sqrt(-2.0 * log(unit53(a)));
    const double ang = 6.283185307179586476925286766559 * unit53(b);
    g0 = rad * cos(ang);
    g1 = rad * sin(ang);
}

// One lane per slot.  sv = sqrt(T / m), sl = sqrt(I T).  Draws: block A's
// first word decides; normals from (A1, A2), (A3, B0), (B1, B2) give v, then L.
__global__ __launch_bounds__(kBlock) void k_thermostat(Sys s, double sv, double sl, double prob,
                                                       uint64_t seed, uint64_t counter) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= s.n) return;
    const uint64_t id = (uint64_t)s.id[q];
    uint64_t A[4] = {id, counter, 0, 0};
    philox4x64_10(A, seed, 0);
    if (!(unit53(A[0]) < prob)) return;
    uint64_t B[4] = {id, counter, 1, 0};
    philox4x64_10(B, seed, 0);
    double g[6];
    box_muller(A[1], A[2], g[0], g[1]);
    box_muller(A[3], B[0], g[2], g[3]);
    box_muller(B[1], B[2], g[4], g[5]);
    s.vel[q] = make_double4(sv * g[0], sv * g[1], sv * g[2], 0.0);
    if (s.pot == 1) s.angm[q] = make_double4(sl * g[3], sl * g[4], sl * g[5], 0.0);
}

hipError_t launch_thermostat(const Sys& s, double sv, double sl, double prob, uint64_t seed,
                             uint64_t counter, hipStream_t st) {
    hipLaunchKernelGGL(k_thermostat, grid_n(s.n), dim3(kBlock), 0, st, s, sv, sl, prob, seed,
                       counter);
    return hipGetLastError();
}

hipError_t launch_count_nonzero(const Sys& s, int prec, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_nonzero, dim3(1), dim3(1), 0, st, s.ctrl);
    const long long waves = (s.max_half + kWave - 1) / kWave;
    const dim3 g((unsigned)std::max(1LL, std::min((waves + 3) / 4, 8192LL)));
    const dim3 b(kBlock);
    if (s.pot == 0) {
        if (prec == 0) hipLaunchKernelGGL((k_count_nonzero<0, 0>), g, b, 0, st, s);
        else hipLaunchKernelGGL((k_count_nonzero<0, 1>), g, b, 0, st, s);
    } else {
        if (prec == 0) hipLaunchKernelGGL((k_count_nonzero<1, 0>), g, b, 0, st, s);
        else hipLaunchKernelGGL((k_count_nonzero<1, 1>), g, b, 0, st, s);
    }
    return hipGetLastError();
}

hipError_t launch_energy(const Sys& s, int prec, hipStream_t st) {
    if (prec == 0) vertex_dispatch<0>(s, false, true, st);
    else if (prec == 1) vertex_dispatch<1>(s, false, true, st);
    else vertex_dispatch<2>(s, false, true, st);
    if (s.pot == 0) hipLaunchKernelGGL(k_kinetic<0>, grid_n(s.n), dim3(kBlock), 0, st, s);
    else hipLaunchKernelGGL(k_kinetic<1>, grid_n(s.n), dim3(kBlock), 0, st, s);
    hipLaunchKernelGGL(k_reduce_partial, dim3(kRedBlocks), dim3(kBlock), 0, st, s);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlocks), 0, st, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forces of coordinates that are already on the device, in one call with no
// caller workspace (md_forces_static): the caller's original-order arrays are
// loaded into the slot records (wrapped into [0, L) as md_set_state wraps
// them), and the slot-order results are stored back in original order.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_fill_zero(int* p, long long n) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) p[k] = 0;
}

// Non-finite or zero input raises ctrl->nonfinite; the record then holds a
// finite stand-in (the origin, the identity rotation) so that every later
// index computation stays in range.
__global__ __launch_bounds__(kBlock) void k_load_records(Sys s, const double* x, const double* q) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    bool ok = true;
    double c[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        double y = x[3 * (size_t)i + k];
        ok = ok && isfinite(y);
        y -= s.box * floor(y / s.box);
        if (y >= s.box) y -= s.box;
        if (y < 0) y += s.box;
        c[k] = isfinite(y) ? y : 0.0;
    }
    const double4 zero = make_double4(0.0, 0.0, 0.0, 0.0);
    s.pos[i] = make_double4(c[0], c[1], c[2], 0.0);
    s.vel[i] = zero;
    s.frc[i] = zero;
    s.id[i] = i;
    if (s.pot != 0) {
        const double* a = q + 4 * (size_t)i;
        const double nn = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
        const bool qok = nn > 0 && isfinite(nn);
        ok = ok && qok;
        s.quat[i] = qok ? make_double4(a[0] / nn, a[1] / nn, a[2] / nn, a[3] / nn)
                        : make_double4(1.0, 0.0, 0.0, 0.0);
        s.angm[i] = zero;
        s.trq[i] = zero;
    }
    if (!ok) atomicOr(&s.ctrl->nonfinite, 1);
}

__global__ __launch_bounds__(kBlock) void k_store_results(Sys s, double* f, double* t) {
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= s.n) return;
    const size_t i = (size_t)s.id[a];
    const double4 F = s.frc[a];
    f[3 * i] = F.x;
    f[3 * i + 1] = F.y;
    f[3 * i + 2] = F.z;
    if (t) {
        const double4 T = s.trq[a];
        t[3 * i] = T.x;
        t[3 * i + 1] = T.y;
        t[3 * i + 2] = T.z;
    }
}

// *out = 0, or the status code of the sticky device error of the call.
__global__ void k_status(const Ctrl* c, int* out, int overflow_code, int nonfinite_code) {
    *out = c->overflow ? overflow_code : (c->nonfinite ? nonfinite_code : 0);
}

hipError_t launch_fill_zero(int* p, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min((n + kBlock - 1) / kBlock, 4096LL);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kBlock), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_load_records(const Sys& s, const double* x, const double* q, hipStream_t st) {
    hipLaunchKernelGGL(k_load_records, grid_n(s.n), dim3(kBlock), 0, st, s, x, q);
    return hipGetLastError();
}

hipError_t launch_store_results(const Sys& s, double* f, double* t, hipStream_t st) {
    hipLaunchKernelGGL(k_store_results, grid_n(s.n), dim3(kBlock), 0, st, s, f, t);
    return hipGetLastError();
}

hipError_t launch_status(const Sys& s, int* out, int overflow_code, int nonfinite_code,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_status, dim3(1), dim3(1), 0, st, s.ctrl, out, overflow_code,
                       nonfinite_code);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched step.  The kernels below run the same bodies as the single-system
// kernels, one system per block: block b of a kernel of class C serves
// (slot, block) = map[C][b].  Idle blocks and slots whose steps for this
// launch are used up return at once.  The descriptor is copied into registers
// once per block, so later stores cannot force it to be reloaded.
// ---------------------------------------------------------------------------

template <int CLS, typename F>
__device__ __forceinline__ void batch_block(const BatchDev& b, int step, F&& body) {
    const int2 m = b.map[CLS][blockIdx.x];
    if (m.x < 0 || step >= b.left[m.x]) return;
    const Sys s = b.tab[m.x];
    body(s, m.y);
}

template <bool ZERO>
__global__ __launch_bounds__(kBlock) void kb_kick_drift(BatchDev b, int step) {
    batch_block<kClsParticle>(b, step, [](const Sys& s, int lb) {
        if (s.pot == 0) b_kick_drift<0, ZERO>(s, lb, s.nblk);
        else b_kick_drift<1, ZERO>(s, lb, s.nblk);
    });
}

__global__ __launch_bounds__(kBlock) void kb_cell_bin(BatchDev b, int step) {
    batch_block<kClsParticle>(b, step, [](const Sys& s, int lb) { b_cell_bin(s, lb, s.nblk); });
}

__global__ __launch_bounds__(kBlock) void kb_cell_scatter(BatchDev b, int step) {
    batch_block<kClsParticle>(b, step, [](const Sys& s, int lb) { b_cell_scatter(s, lb, s.nblk); });
}

__global__ __launch_bounds__(kBlock) void kb_sort_tiles(BatchDev b, int step) {
    batch_block<kClsSortTiles>(b, step, [](const Sys& s, int lb) {
        b_sort_tiles(s, lb, class_blocks(s, kClsSortTiles));
    });
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void kb_build(BatchDev b, int step) {
    batch_block<kClsParticle>(b, step, [](const Sys& s, int lb) { b_build(s, lb, s.nblk); });
}

__global__ __launch_bounds__(kBlock) void kb_half_fill(BatchDev b, int step) {
    batch_block<kClsTile>(b, step, [](const Sys& s, int lb) { b_half_fill(s, lb, s.ntiles); });
}

// Vertex forces with the closing half kick, dispatched per block on the
// system's potential and precision (uniform branches).
template <int C>
__global__ __launch_bounds__(kBlock) void kb_vertex(BatchDev b, int step) {
    batch_block<C>(b, step, [](const Sys& s, int lb) {
        constexpr int T = kTileTpp;
        if (s.pot == 0) {
            if (s.prec == 0) b_vertex_lj<0, T, true, false>(s, lb, s.ntiles);
            else if (s.prec == 1) b_vertex_lj<1, T, true, false>(s, lb, s.ntiles);
            else b_vertex_lj<2, T, true, false>(s, lb, s.ntiles);
        } else {
            const int nb = class_blocks(s, kClsVertex0 + lds_bucket(s));
            if (patchy_vertex_tpp(s) > 1) {
                if (s.prec == 0) b_vertex_patchy<0, true, false, T>(s, lb, nb);
                else if (s.prec == 1) b_vertex_patchy<1, true, false, T>(s, lb, nb);
                else b_vertex_patchy<2, true, false, T>(s, lb, nb);
            } else {
                if (s.prec == 0) b_vertex_patchy<0, true, false, 1>(s, lb, nb);
                else if (s.prec == 1) b_vertex_patchy<1, true, false, 1>(s, lb, nb);
                else b_vertex_patchy<2, true, false, 1>(s, lb, nb);
            }
        }
    });
}

// Deterministic edge mode: the edge indices of the full-list entries (after
// the half list), the per-edge store pass (grid-stride over the system's
// half list with the class's blocks) and the ordered gather.
__global__ __launch_bounds__(kBlock) void kb_col_fill(BatchDev b, int step) {
    batch_block<kClsTile>(b, step, [](const Sys& s, int lb) { b_col_fill(s, lb, s.ntiles); });
}

template <int C>
__global__ __launch_bounds__(kBlock) void kb_edge_store(BatchDev b, int step) {
    batch_block<C>(b, step, [](const Sys& s, int lb) {
        const int nb = class_blocks(s, C);
        if (s.pot == 0) {
            if (s.prec == 0) b_edge<0, 0, true>(s, lb, nb);
            else b_edge<0, 1, true>(s, lb, nb);
        } else {
            if (s.prec == 0) b_edge<1, 0, true>(s, lb, nb);
            else b_edge<1, 1, true>(s, lb, nb);
        }
    });
}

__global__ __launch_bounds__(kBlock) void kb_edge_gather(BatchDev b, int step) {
    batch_block<kClsTile>(b, step, [](const Sys& s, int lb) {
        if (s.pot == 0) b_edge_gather<0>(s, lb, s.ntiles);
        else b_edge_gather<1>(s, lb, s.ntiles);
    });
}

template <int C>
__global__ __launch_bounds__(kBlock) void kb_edge(BatchDev b, int step) {
    batch_block<C>(b, step, [](const Sys& s, int lb) {
        if (s.pot == 0) {
            constexpr bool stage = edge_stages_positions(bucket_cap(C - kClsEdge0));
            if (s.prec == 0) b_edge_lj_tile<0, stage>(s, lb, s.ntiles);
            else b_edge_lj_tile<1, stage>(s, lb, s.ntiles);
        } else if (patchy_edge_by_tile(s)) {
            constexpr bool acc = patchy_edge_accumulates(bucket_cap(C - kClsEdge0));
            if (s.prec == 0) b_edge_patchy_tile<0, acc>(s, lb);
            else b_edge_patchy_tile<1, acc>(s, lb);
        } else {
            if (s.prec == 0) b_edge<1, 0>(s, lb, s.ntiles);
            else b_edge<1, 1>(s, lb, s.ntiles);
        }
    });
}

// PLANES: after the atomic edge pass, whose LJ forces are in the planes.
template <bool PLANES>
__global__ __launch_bounds__(kBlock) void kb_kick(BatchDev b, int step) {
    batch_block<kClsParticle>(b, step, [](const Sys& s, int lb) {
        if (s.pot == 0) b_kick<0, PLANES>(s, lb, s.nblk);
        else b_kick<1>(s, lb, s.nblk);
    });
}

// Closes a launch of `steps` steps: every slot's budget drops by what it ran.
__global__ __launch_bounds__(kBlock) void kb_advance(BatchDev b, int steps) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < b.nslots) b.left[i] = max(0, b.left[i] - steps);
}

hipError_t launch_batch_steps(const BatchDev& b, const int* grid, int mode, int steps,
                              hipStream_t st) {
    const dim3 blk(kBlock);
    auto g = [&](int cls) { return dim3((unsigned)grid[cls]); };
    // one launch per LDS bucket in use, each with that bucket's LDS
    auto per_bucket = [&](auto launch) {
        launch(std::integral_constant<int, 0>{});
        launch(std::integral_constant<int, 1>{});
        launch(std::integral_constant<int, 2>{});
    };
    const size_t sh_map = sizeof(int) * (size_t)(kLdsCapMax + 8);
    for (int k = 0; k < steps; k++) {
        // the passes that add into F with atomics need it cleared
        if (mode == 1) hipLaunchKernelGGL(kb_kick_drift<true>, g(kClsParticle), blk, 0, st, b, k);
        else hipLaunchKernelGGL(kb_kick_drift<false>, g(kClsParticle), blk, 0, st, b, k);
        hipLaunchKernelGGL(kb_cell_bin, g(kClsParticle), blk, 0, st, b, k);
        hipLaunchKernelGGL(kb_cell_scatter, g(kClsParticle), blk, 0, st, b, k);
        hipLaunchKernelGGL(kb_sort_tiles, g(kClsSortTiles), blk, 0, st, b, k);
        hipLaunchKernelGGL(kb_build, g(kClsParticle), blk, 0, st, b, k);
        if (mode == 0) {
            per_bucket([&](auto bk) {
                constexpr int B = decltype(bk)::value;
                if (grid[kClsVertex0 + B] > 0)
                    hipLaunchKernelGGL(kb_vertex<kClsVertex0 + B>, g(kClsVertex0 + B), blk,
                                       lds_region_bytes(bucket_cap(B)), st, b, k);
            });
        } else if (mode == 3) {  // deterministic edge: per-edge records, ordered gather
            hipLaunchKernelGGL(kb_half_fill, g(kClsTile), blk, sh_map, st, b, k);
            hipLaunchKernelGGL(kb_col_fill, g(kClsTile), blk, sh_map, st, b, k);
            per_bucket([&](auto bk) {
                constexpr int B = decltype(bk)::value;
                if (grid[kClsEdge0 + B] > 0)
                    hipLaunchKernelGGL(kb_edge_store<kClsEdge0 + B>, g(kClsEdge0 + B), blk, 0, st, b, k);
            });
            hipLaunchKernelGGL(kb_edge_gather, g(kClsTile), blk, 0, st, b, k);
            hipLaunchKernelGGL(kb_kick<false>, g(kClsParticle), blk, 0, st, b, k);
        } else {
            hipLaunchKernelGGL(kb_half_fill, g(kClsTile), blk, sh_map, st, b, k);
            per_bucket([&](auto bk) {
                constexpr int B = decltype(bk)::value;
                // the larger of the LJ and patchy passes' LDS
                constexpr int cap = bucket_cap(B);
                const size_t sh = std::max(edge_lds_bytes(cap), patchy_edge_lds_bytes(cap));
                if (grid[kClsEdge0 + B] > 0)
                    hipLaunchKernelGGL(kb_edge<kClsEdge0 + B>, g(kClsEdge0 + B), blk, sh, st, b, k);
            });
            hipLaunchKernelGGL(kb_kick<true>, g(kClsParticle), blk, 0, st, b, k);
        }
    }
    hipLaunchKernelGGL(kb_advance, dim3((b.nslots + kBlock - 1) / kBlock), blk, 0, st, b, steps);
    return hipGetLastError();
}

int batch_kernel_class(const void* func) {
    const void* particle[] = {reinterpret_cast<const void*>(&kb_kick_drift<false>),
                              reinterpret_cast<const void*>(&kb_kick_drift<true>),
                              reinterpret_cast<const void*>(&kb_cell_bin),
                              reinterpret_cast<const void*>(&kb_cell_scatter),
                              reinterpret_cast<const void*>(&kb_build),
                              reinterpret_cast<const void*>(&kb_kick<false>),
                              reinterpret_cast<const void*>(&kb_kick<true>)};
    for (const void* f : particle)
        if (f == func) return kClsParticle;
    if (func == reinterpret_cast<const void*>(&kb_sort_tiles)) return kClsSortTiles;
    if (func == reinterpret_cast<const void*>(&kb_half_fill) ||
        func == reinterpret_cast<const void*>(&kb_col_fill) ||
        func == reinterpret_cast<const void*>(&kb_edge_gather))
        return kClsTile;
    if (func == reinterpret_cast<const void*>(&kb_edge_store<kClsEdge0>)) return kClsEdge0;
    if (func == reinterpret_cast<const void*>(&kb_edge_store<kClsEdge1>)) return kClsEdge1;
    if (func == reinterpret_cast<const void*>(&kb_edge_store<kClsEdge2>)) return kClsEdge2;
    if (func == reinterpret_cast<const void*>(&kb_vertex<kClsVertex0>)) return kClsVertex0;
    if (func == reinterpret_cast<const void*>(&kb_vertex<kClsVertex1>)) return kClsVertex1;
    if (func == reinterpret_cast<const void*>(&kb_vertex<kClsVertex2>)) return kClsVertex2;
    if (func == reinterpret_cast<const void*>(&kb_edge<kClsEdge0>)) return kClsEdge0;
    if (func == reinterpret_cast<const void*>(&kb_edge<kClsEdge1>)) return kClsEdge1;
    if (func == reinterpret_cast<const void*>(&kb_edge<kClsEdge2>)) return kClsEdge2;
    if (func == reinterpret_cast<const void*>(&kb_advance)) return -1;
    return -2;
}


}  // namespace md
