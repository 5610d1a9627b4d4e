// HIP kernels for gfx950: cell-list counting sort, Verlet-list build,
// vertex and edge pair-force decompositions, velocity-Verlet integration and
// deterministic energy reduction.
//
// Layout: particle records are packed 32-byte double4 (x, y, z, unused) in
// cell-sorted slot order, so one neighbour gather touches one 32-byte sector;
// the full Verlet list is ELL column-major (nbr[k * n + i]) so that the k-th
// entries of consecutive particles are consecutive words (coalesced); the half
// list is CSR by row.  No kernel here uses matrix cores: the pair step is a
// gather plus a short scalar formula per pair, not a dense contraction.
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

__device__ __forceinline__ int cell_coord(double x, double cell_inv, int nc) {
    int c = (int)(x * cell_inv);
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}

__device__ __forceinline__ double* comp(double4* a, int i) { return reinterpret_cast<double*>(a + i); }

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

// The four tetrahedral patch directions of a particle with orientation
// q = (w, x, y, z): u_a = R(q) e_a with e_a = (+-1, +-1, +-1)/sqrt(3) having an
// even number of minus signs, i.e. sums and differences of R's columns.
template <typename R>
__device__ __forceinline__ void patch_dirs(const double4& q, V3<R> u[4]) {
    R w = (R)q.x, x = (R)q.y, y = (R)q.z, z = (R)q.w;
    V3<R> c0 = {R(1) - R(2) * (y * y + z * z), R(2) * (x * y + w * z), R(2) * (x * z - w * y)};
    V3<R> c1 = {R(2) * (x * y - w * z), R(1) - R(2) * (x * x + z * z), R(2) * (y * z + w * x)};
    V3<R> c2 = {R(2) * (x * z + w * y), R(2) * (y * z - w * x), R(1) - R(2) * (x * x + y * y)};
    const R k = R(0.57735026918962576451);  // 1/sqrt(3)
    u[0] = {k * (c0.x + c1.x + c2.x), k * (c0.y + c1.y + c2.y), k * (c0.z + c1.z + c2.z)};
    u[1] = {k * (c0.x - c1.x - c2.x), k * (c0.y - c1.y - c2.y), k * (c0.z - c1.z - c2.z)};
    u[2] = {k * (-c0.x + c1.x - c2.x), k * (-c0.y + c1.y - c2.y), k * (-c0.z + c1.z - c2.z)};
    u[3] = {k * (-c0.x - c1.x + c2.x), k * (-c0.y - c1.y + c2.y), k * (-c0.z - c1.z + c2.z)};
}

__device__ __forceinline__ float exp_r(float a) { return __expf(a); }
__device__ __forceinline__ double exp_r(double a) { return exp(a); }

// Patchy pair: WCA core + sum over facing patch pairs of
// -eps_p exp(-|d_ab|^2 / w^2) * A(c_i^a) * A(c_j^b), A(c) = c^2 for c > 0.
// d = x_j - x_i (minimum image), r2 = |d|^2 < r_cut^2.  Outputs the force on j
// (fj, the force on i is -fj), the torques on i and j, and the pair energy.
// Torques come from the patch-vector gradients: tau = sum_a u_a x (-dV/du_a).
template <typename R>
__device__ __forceinline__ void patchy_pair(const V3<R>& d, R r2, const V3<R> ui[4],
                                            const V3<R> uj[4], const PatchyC<R>& c,
                                            V3<R>& fj, V3<R>& ti, V3<R>& tj, R& v) {
    fj = {0, 0, 0};
    ti = {0, 0, 0};
    tj = {0, 0, 0};
    v = 0;
    if (r2 < c.wca2) {
        R inv = R(1) / r2;
        R s2 = c.sig2 * inv;
        R s6 = s2 * s2 * s2;
        v += c.eps4 * (s6 * s6 - s6) + c.eps;
        R fr = c.eps24 * (R(2) * s6 * s6 - s6) * inv;
        fj.x += fr * d.x;
        fj.y += fr * d.y;
        fj.z += fr * d.z;
    }
    R rinv = R(1) / sqrt(r2);
    V3<R> h = {d.x * rinv, d.y * rinv, d.z * rinv};
    R ci[4], cj[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        ci[a] = dot3(ui[a], h);
        cj[a] = -dot3(uj[a], h);
    }
#pragma unroll
    for (int a = 0; a < 4; a++) {
        if (!(ci[a] > R(0))) continue;
        R Ai = ci[a] * ci[a];
#pragma unroll
        for (int b = 0; b < 4; b++) {
            if (!(cj[b] > R(0))) continue;
            R Aj = cj[b] * cj[b];
            V3<R> dd = {d.x + c.delta * (uj[b].x - ui[a].x), d.y + c.delta * (uj[b].y - ui[a].y),
                        d.z + c.delta * (uj[b].z - ui[a].z)};
            R s2 = dot3(dd, dd);
            if (c.rpc2 > R(0) && !(s2 < c.rpc2)) continue;
            R g = -c.eps_p * exp_r(-s2 * c.inv_w2);
            R G = g * Ai * Aj;
            v += G;
            // gradient pieces: Gaussian (along d_ab) and the two cosines
            R kd = R(2) * G * c.inv_w2;           // -dG/d(d_ab) = -kd... see below
            R ki = g * Aj * R(2) * ci[a] * rinv;  // d/dr through c_i
            R kj = g * Ai * R(2) * cj[b] * rinv;  // d/dr through c_j
            // dV/dr = -kd d_ab + ki (u_i - c_i h) + kj (-u_j - c_j h); F_j = -dV/dr
            fj.x += kd * dd.x - ki * (ui[a].x - ci[a] * h.x) + kj * (uj[b].x + cj[b] * h.x);
            fj.y += kd * dd.y - ki * (ui[a].y - ci[a] * h.y) + kj * (uj[b].y + cj[b] * h.y);
            fj.z += kd * dd.z - ki * (ui[a].z - ci[a] * h.z) + kj * (uj[b].z + cj[b] * h.z);
            // -dV/du_i = -(delta kd d_ab + ki r h),  -dV/du_j = delta kd d_ab + kj r h
            R r = r2 * rinv;
            V3<R> mi = {-(c.delta * kd * dd.x + ki * r * h.x), -(c.delta * kd * dd.y + ki * r * h.y),
                        -(c.delta * kd * dd.z + ki * r * h.z)};
            V3<R> mj = {c.delta * kd * dd.x + kj * r * h.x, c.delta * kd * dd.y + kj * r * h.y,
                        c.delta * kd * dd.z + kj * r * h.z};
            ti.x += ui[a].y * mi.z - ui[a].z * mi.y;
            ti.y += ui[a].z * mi.x - ui[a].x * mi.z;
            ti.z += ui[a].x * mi.y - ui[a].y * mi.x;
            tj.x += uj[b].y * mj.z - uj[b].z * mj.y;
            tj.y += uj[b].z * mj.x - uj[b].x * mj.z;
            tj.z += uj[b].x * mj.y - uj[b].y * mj.x;
        }
    }
}

template <typename R>
__device__ __forceinline__ const PatchyC<R>& pick(const PatchyC<double>& a, const PatchyC<float>& b);
template <>
__device__ __forceinline__ const PatchyC<double>& pick<double>(const PatchyC<double>& a,
                                                               const PatchyC<float>&) {
    return a;
}
template <>
__device__ __forceinline__ const PatchyC<float>& pick<float>(const PatchyC<double>&,
                                                             const PatchyC<float>& b) {
    return b;
}

// ---------------------------------------------------------------------------
// Control
// ---------------------------------------------------------------------------

__global__ void k_set_rebuild(Ctrl* c) { c->rebuild = 1; }

__global__ void k_clear_ctrl(Ctrl* c) {
    c->rebuild = 0;
    c->overflow = 0;
    c->nonfinite = 0;
    c->max_count = 0;
    c->npairs = 0;
    c->rebuilds = 0;
}

// ---------------------------------------------------------------------------
// Cell-list counting sort.  Every kernel returns at once unless a rebuild is
// due, so the sequence can sit in every step without a host round trip.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_cell_bin(Sys s) {
    if (!s.ctrl->rebuild) return;
    int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= s.n) return;
    double4 x = s.pos[p];
    int cx = cell_coord(x.x, s.cell_inv, s.nc);
    int cy = cell_coord(x.y, s.cell_inv, s.nc);
    int cz = cell_coord(x.z, s.cell_inv, s.nc);
    int c = (cz * s.nc + cy) * s.nc + cx;
    s.cell[p] = c;
    s.rank[p] = atomicAdd(&s.ccount[c], 1);
}

// One workgroup: exclusive scan of the cell counts into cell_start, then the
// counts are cleared for the next build.
__global__ __launch_bounds__(kScanThreads) void k_cell_scan(Sys s) {
    if (!s.ctrl->rebuild) return;
    __shared__ int sh[kScanThreads];
    int t = threadIdx.x;
    int per = (s.ncell + kScanThreads - 1) / kScanThreads;
    int b = t * per;
    int e = min(b + per, s.ncell);
    int sum = 0;
    for (int k = b; k < e; k++) sum += s.ccount[k];
    sh[t] = sum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int run = sh[t] - sum;
    for (int k = b; k < e; k++) {
        int c = s.ccount[k];
        s.cstart[k] = run;
        run += c;
        s.ccount[k] = 0;
    }
    if (t == kScanThreads - 1) s.cstart[s.ncell] = sh[t];
    if (t == 0) s.ctrl->max_count = 0;  // the list build that follows records its maximum
}

__global__ __launch_bounds__(kBlock) void k_cell_scatter(Sys s) {
    if (!s.ctrl->rebuild) return;
    int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= s.n) return;
    s.order[s.cstart[s.cell[p]] + s.rank[p]] = p;
}

// One thread per cell: order the cell's members by original id, so that the
// slot order (and every sum over a list) does not depend on atomic timing.
__global__ __launch_bounds__(kBlock) void k_cell_sort(Sys s) {
    if (!s.ctrl->rebuild) return;
    int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= s.ncell) return;
    int b = s.cstart[c], e = s.cstart[c + 1];
    for (int k = b + 1; k < e; k++) {
        int p = s.order[k];
        int key = s.id[p];
        int m = k - 1;
        while (m >= b && s.id[s.order[m]] > key) {
            s.order[m + 1] = s.order[m];
            m--;
        }
        s.order[m + 1] = p;
    }
}

__global__ __launch_bounds__(kBlock) void k_reorder(Sys s) {
    if (!s.ctrl->rebuild) return;
    int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= s.n) return;
    int p = s.order[k];
    s.tpos[k] = s.pos[p];
    s.tvel[k] = s.vel[p];
    s.tid[k] = s.id[p];
    if (s.pot == 1) {
        s.tquat[k] = s.quat[p];
        s.tangm[k] = s.angm[p];
    }
}

// ---------------------------------------------------------------------------
// Verlet-list build.  One thread per particle (slot i) scans the 27 cells
// around its own (all cells of a dimension when fewer than three fit) and
// keeps every j != i with r_ij^2 < r_v^2 in FP64.  It also moves its particle
// record from the reorder buffer back into the state and stores the build
// reference position.  Per-block totals of the half-list lengths feed the
// half-list offsets.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_build(Sys s) {
    if (!s.ctrl->rebuild) return;
    __shared__ int red[kBlock / kWave];
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    int i = lb * kBlock + threadIdx.x;
    int half = 0;
    if (i < s.n) {
        double4 xi = s.tpos[i];
        s.pos[i] = xi;
        s.xbuild[i] = xi;
        s.vel[i] = s.tvel[i];
        s.id[i] = s.tid[i];
        if (s.pot == 1) {
            s.quat[i] = s.tquat[i];
            s.angm[i] = s.tangm[i];
        }
        int nc = s.nc;
        int cx = cell_coord(xi.x, s.cell_inv, nc);
        int cy = cell_coord(xi.y, s.cell_inv, nc);
        int cz = cell_coord(xi.z, s.cell_inv, nc);
        int span = nc >= 3 ? 3 : nc;   // distinct cells per dimension
        int lo = nc >= 3 ? -1 : 0;
        int count = 0;
        for (int dz = 0; dz < span; dz++) {
            int az = cz + lo + dz;
            az = az < 0 ? az + nc : (az >= nc ? az - nc : az);
            for (int dy = 0; dy < span; dy++) {
                int ay = cy + lo + dy;
                ay = ay < 0 ? ay + nc : (ay >= nc ? ay - nc : ay);
                for (int dx = 0; dx < span; dx++) {
                    int ax = cx + lo + dx;
                    ax = ax < 0 ? ax + nc : (ax >= nc ? ax - nc : ax);
                    int c = (az * nc + ay) * nc + ax;
                    int e = s.cstart[c + 1];
                    for (int j = s.cstart[c]; j < e; j++) {
                        if (j == i) continue;
                        double4 xj = s.tpos[j];
                        double ddx = wrap_delta(xj.x - xi.x, s.box, s.inv_box);
                        double ddy = wrap_delta(xj.y - xi.y, s.box, s.inv_box);
                        double ddz = wrap_delta(xj.z - xi.z, s.box, s.inv_box);
                        double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        if (r2 < s.rv2) {
                            if (count < s.cap) {
                                s.nbr[(size_t)count * s.n + i] = j;
                                half += (j > i);
                            }
                            count++;
                        }
                    }
                }
            }
        }
        s.ncount[i] = count < s.cap ? count : s.cap;
        s.hcount[i] = half;
        if (count > s.cap) atomicOr(&s.ctrl->overflow, 1);
        atomicMax(&s.ctrl->max_count, count);
    }
    // block total of half-list lengths
    int v = half;
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / kWave; w++) t += red[w];
        s.bsum[lb] = t;
    }
}

// One workgroup: exclusive scan of the per-block half totals.
__global__ __launch_bounds__(kScanThreads) void k_half_scan(Sys s) {
    if (!s.ctrl->rebuild) return;
    __shared__ long long sh[kScanThreads];
    int t = threadIdx.x;
    int per = (s.nblk + kScanThreads - 1) / kScanThreads;
    int b = t * per;
    int e = min(b + per, s.nblk);
    long long sum = 0;
    for (int k = b; k < e; k++) sum += s.bsum[k];
    sh[t] = sum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        long long v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    long long run = sh[t] - sum;
    for (int k = b; k < e; k++) {
        int c = s.bsum[k];
        s.bsum[k] = (int)(run < s.max_half ? run : s.max_half);
        run += c;
    }
    if (t == kScanThreads - 1) {
        long long tot = sh[t];
        s.ctrl->npairs = tot < s.max_half ? tot : s.max_half;
        if (tot > s.max_half) atomicOr(&s.ctrl->overflow, 1);
        s.ctrl->rebuilds += 1;
    }
}

// Same blocking as k_build: block-local exclusive scan of the half lengths plus
// the block offset gives each row's start; the row then copies its j > i
// entries into the CSR half list and records the chunk heads (first row of
// every 64-entry chunk) that the edge kernel uses to find its rows.
__global__ __launch_bounds__(kBlock) void k_half_fill(Sys s) {
    if (!s.ctrl->rebuild) return;
    __shared__ int sh[kBlock];
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    int t = threadIdx.x;
    int i = lb * kBlock + t;
    int h = i < s.n ? s.hcount[i] : 0;
    sh[t] = h;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    if (i >= s.n) return;
    long long start = (long long)s.bsum[lb] + sh[t] - h;
    long long cap = s.max_half;
    if (start > cap) start = cap;
    s.hstart[i] = (int)start;
    long long end = start + h;
    if (end > cap) end = cap;
    if (i == s.n - 1) s.hstart[s.n] = (int)end;
    long long k = start;
    int cnt = s.ncount[i];
    for (int m = 0; m < cnt && k < end; m++) {
        int j = s.nbr[(size_t)m * s.n + i];
        if (j > i) s.hj[k++] = j;
    }
    for (long long c0 = (start + kWave - 1) / kWave * kWave; c0 < end; c0 += kWave)
        s.chunk_row[c0 / kWave] = i;
}

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
};

template <int PREC, bool KICK, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_vertex_lj(Sys s) {
    const LJc<double>& c64 = s.l64;
    const LJc<float>& c32 = s.l32;
    using R = typename std::conditional<PREC == 0, double, float>::type;
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    int i = lb * kBlock + threadIdx.x;
    if (KICK && blockIdx.x == 0 && threadIdx.x == 0) s.ctrl->rebuild = 0;
    if (i >= s.n) return;
    double4 xi = s.pos[i];
    int cnt = s.ncount[i];
    Acc3<PREC> f;
    double e = 0, w = 0;
    const int* nb = s.nbr + i;
    for (int k = 0; k < cnt; k++) {
        int j = nb[(size_t)k * s.n];
        double4 xj = s.pos[j];
        double dx = wrap_delta(xj.x - xi.x, s.box, s.inv_box);
        double dy = wrap_delta(xj.y - xi.y, s.box, s.inv_box);
        double dz = wrap_delta(xj.z - xi.z, s.box, s.inv_box);
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < s.rc2) {
            if (PREC == 0) {
                double v;
                double fr = lj_fr<double>(r2, c64, ENERGY ? &v : nullptr);
                f.add(-fr * dx, -fr * dy, -fr * dz);
                if (ENERGY) {
                    e += 0.5 * v;
                    w += 0.5 * fr * r2;
                }
            } else {
                float v;
                float fr = lj_fr<float>((float)r2, c32, ENERGY ? &v : nullptr);
                f.add(-fr * (float)dx, -fr * (float)dy, -fr * (float)dz);
                if (ENERGY) {
                    e += 0.5 * (double)v;
                    w += 0.5 * (double)fr * r2;
                }
            }
        }
    }
    double fx = f.x, fy = f.y, fz = f.z;
    if (ENERGY) {  // energy pass: leaves the forces of the last force pass alone
        s.epart[i] = e;
        s.wpart[i] = w;
        return;
    }
    s.frc[i] = make_double4(fx, fy, fz, 0.0);
    if (!isfinite(fx + fy + fz)) atomicOr(&s.ctrl->nonfinite, 1);
    if (KICK) {
        double4 v = s.vel[i];
        v.x += s.hdt * fx * s.inv_mass;
        v.y += s.hdt * fy * s.inv_mass;
        v.z += s.hdt * fz * s.inv_mass;
        s.vel[i] = v;
    }
}

template <int PREC, bool KICK, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_vertex_patchy(Sys s) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    int i = lb * kBlock + threadIdx.x;
    if (KICK && blockIdx.x == 0 && threadIdx.x == 0) s.ctrl->rebuild = 0;
    if (i >= s.n) return;
    const PatchyC<R>& c = pick<R>(s.p64, s.p32);
    double4 xi = s.pos[i];
    V3<R> ui[4];
    patch_dirs<R>(s.quat[i], ui);
    int cnt = s.ncount[i];
    Acc3<PREC> f, t;
    double e = 0, w = 0;
    const int* nb = s.nbr + i;
    for (int k = 0; k < cnt; k++) {
        int j = nb[(size_t)k * s.n];
        double4 xj = s.pos[j];
        double dx = wrap_delta(xj.x - xi.x, s.box, s.inv_box);
        double dy = wrap_delta(xj.y - xi.y, s.box, s.inv_box);
        double dz = wrap_delta(xj.z - xi.z, s.box, s.inv_box);
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < s.rc2) {
            V3<R> uj[4];
            patch_dirs<R>(s.quat[j], uj);
            V3<R> d = {(R)dx, (R)dy, (R)dz};
            V3<R> fj, ti, tj;
            R v;
            patchy_pair<R>(d, (R)r2, ui, uj, c, fj, ti, tj, v);
            f.add(-fj.x, -fj.y, -fj.z);
            t.add(ti.x, ti.y, ti.z);
            if (ENERGY) {
                e += 0.5 * (double)v;
                w += 0.5 * ((double)fj.x * dx + (double)fj.y * dy + (double)fj.z * dz);
            }
        }
    }
    double fx = f.x, fy = f.y, fz = f.z;
    double tx = t.x, ty = t.y, tz = t.z;
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

template <int POT, int PREC>
__global__ __launch_bounds__(kBlock) void k_edge(Sys s) {
    using R = typename std::conditional<PREC == 0, double, float>::type;
    const long long npairs = s.ctrl->npairs;
    const long long nchunks = (npairs + kWave - 1) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const long long nw = (long long)gridDim.x * (kBlock / kWave);
    const long long w0 = (long long)xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) +
                         threadIdx.x / kWave;
    double* F = reinterpret_cast<double*>(s.frc);
    double* T = reinterpret_cast<double*>(s.trq);
    for (long long m = w0; m < nchunks; m += nw) {
        const int r0 = s.chunk_row[m];
        const int rlast = (m + 1 < nchunks) ? s.chunk_row[m + 1] : s.n - 1;
        const long long e = m * kWave + lane;
        const bool valid = e < npairs;
        // row of entry e: r0 plus the number of later row starts <= e
        int row = r0;
        for (int base = r0 + 1; base <= rlast; base += kWave) {
            int rr = base + lane;
            int hs = rr <= rlast ? s.hstart[rr] : INT_MAX;
            int lim = min(kWave, rlast - base + 1);
            for (int q = 0; q < lim; q++) row += (__builtin_amdgcn_readlane(hs, q) <= e);
        }
        const int i = row;
        const int j = valid ? s.hj[e] : i;
        double fx = 0, fy = 0, fz = 0, tix = 0, tiy = 0, tiz = 0, tjx = 0, tjy = 0, tjz = 0;
        if (valid) {
            double4 xi = s.pos[i], xj = s.pos[j];
            double dx = wrap_delta(xj.x - xi.x, s.box, s.inv_box);
            double dy = wrap_delta(xj.y - xi.y, s.box, s.inv_box);
            double dz = wrap_delta(xj.z - xi.z, s.box, s.inv_box);
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
                    const PatchyC<R>& c = pick<R>(s.p64, s.p32);
                    V3<R> ui[4], uj[4];
                    patch_dirs<R>(s.quat[i], ui);
                    patch_dirs<R>(s.quat[j], uj);
                    V3<R> d = {(R)dx, (R)dy, (R)dz};
                    V3<R> fj, ti, tj;
                    R v;
                    patchy_pair<R>(d, (R)r2, ui, uj, c, fj, ti, tj, v);
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
        const bool nz = (fx != 0.0) | (fy != 0.0) | (fz != 0.0) | (tix != 0.0) | (tiy != 0.0) |
                        (tiz != 0.0) | (tjx != 0.0) | (tjy != 0.0) | (tjz != 0.0);
        // j side: only non-zero pairs touch memory
        if (nz) {
            unsafeAtomicAdd(F + 4 * (size_t)j + 0, fx);
            unsafeAtomicAdd(F + 4 * (size_t)j + 1, fy);
            unsafeAtomicAdd(F + 4 * (size_t)j + 2, fz);
            if (POT == 1) {
                unsafeAtomicAdd(T + 4 * (size_t)j + 0, tjx);
                unsafeAtomicAdd(T + 4 * (size_t)j + 1, tjy);
                unsafeAtomicAdd(T + 4 * (size_t)j + 2, tjz);
            }
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
            bool rnz = (sx != 0.0) | (sy != 0.0) | (sz != 0.0) | (ux != 0.0) | (uy != 0.0) |
                       (uz != 0.0);
            if (head && rnz) {
                unsafeAtomicAdd(F + 4 * (size_t)i + 0, sx);
                unsafeAtomicAdd(F + 4 * (size_t)i + 1, sy);
                unsafeAtomicAdd(F + 4 * (size_t)i + 2, sz);
                if (POT == 1) {
                    unsafeAtomicAdd(T + 4 * (size_t)i + 0, ux);
                    unsafeAtomicAdd(T + 4 * (size_t)i + 1, uy);
                    unsafeAtomicAdd(T + 4 * (size_t)i + 2, uz);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Velocity Verlet (FP64).  kick_drift: v += dt/2 F/m, x += dt v, wrap into
// [0, L); patchy also L += dt/2 tau and a free rotation of q by |L|/I dt
// about L.  Flags a rebuild if any particle moved more than skin/2 since the
// last build.  Optionally zeroes F (and tau) for the edge pass.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wrap_pos(double y, double L) {
    if (y >= L) y -= L;
    if (y < 0) y += L;
    return y;
}

template <int POT, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_kick_drift(Sys s) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    double4 f = s.frc[i];
    double4 v = s.vel[i];
    double4 x = s.pos[i];
    v.x += s.hdt * f.x * s.inv_mass;
    v.y += s.hdt * f.y * s.inv_mass;
    v.z += s.hdt * f.z * s.inv_mass;
    x.x = wrap_pos(x.x + s.dt * v.x, s.box);
    x.y = wrap_pos(x.y + s.dt * v.y, s.box);
    x.z = wrap_pos(x.z + s.dt * v.z, s.box);
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
    if (ZERO) s.frc[i] = make_double4(0, 0, 0, 0);
    double4 xb = s.xbuild[i];
    double ddx = wrap_delta(x.x - xb.x, s.box, s.inv_box);
    double ddy = wrap_delta(x.y - xb.y, s.box, s.inv_box);
    double ddz = wrap_delta(x.z - xb.z, s.box, s.inv_box);
    if (ddx * ddx + ddy * ddy + ddz * ddz > s.disp2) s.ctrl->rebuild = 1;
}

template <int POT>
__global__ __launch_bounds__(kBlock) void k_kick(Sys s) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) s.ctrl->rebuild = 0;
    if (i >= s.n) return;
    double4 f = s.frc[i];
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

__global__ __launch_bounds__(kBlock) void k_zero_forces(Sys s) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    s.frc[i] = make_double4(0, 0, 0, 0);
    if (s.pot == 1) s.trq[i] = make_double4(0, 0, 0, 0);
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
    hipLaunchKernelGGL(k_clear_ctrl, dim3(1), dim3(1), 0, st, s.ctrl);
    return hipGetLastError();
}

hipError_t launch_rebuild(const Sys& s, hipStream_t st, bool cells, bool lists) {
    if (cells) {
        hipLaunchKernelGGL(k_cell_bin, grid_n(s.n), dim3(kBlock), 0, st, s);
        hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(kScanThreads), 0, st, s);
        hipLaunchKernelGGL(k_cell_scatter, grid_n(s.n), dim3(kBlock), 0, st, s);
        hipLaunchKernelGGL(k_cell_sort, grid_n(s.ncell), dim3(kBlock), 0, st, s);
        hipLaunchKernelGGL(k_reorder, grid_n(s.n), dim3(kBlock), 0, st, s);
    }
    if (lists) {
        hipLaunchKernelGGL(k_build, dim3(s.nblk), dim3(kBlock), 0, st, s);
        hipLaunchKernelGGL(k_half_scan, dim3(1), dim3(kScanThreads), 0, st, s);
        hipLaunchKernelGGL(k_half_fill, dim3(s.nblk), dim3(kBlock), 0, st, s);
    }
    return hipGetLastError();
}

void set_potential(Sys& s, double eps, double sigma, double rc, double eps_p, double w,
                   double delta, double rpc) {
    double s2 = sigma * sigma / (rc * rc);
    double s6 = s2 * s2 * s2;
    double vs = 4.0 * eps * (s6 * s6 - s6);
    s.l64 = {sigma * sigma, 4.0 * eps, 24.0 * eps, rc * rc, vs};
    s.l32 = {(float)(sigma * sigma), (float)(4.0 * eps), (float)(24.0 * eps), (float)(rc * rc),
             (float)vs};
    double wca2 = cbrt(2.0) * sigma * sigma;
    double rpc2 = rpc > 0 ? rpc * rpc : 0.0;
    s.p64 = {sigma * sigma, 4.0 * eps, 24.0 * eps, eps, wca2, eps_p, 1.0 / (w * w), delta, rpc2};
    s.p32 = {(float)(sigma * sigma), (float)(4.0 * eps), (float)(24.0 * eps), (float)eps,
             (float)wca2, (float)eps_p, (float)(1.0 / (w * w)), (float)delta, (float)rpc2};
}

template <int PREC>
static void vertex_dispatch(const Sys& s, bool kick, bool energy, hipStream_t st) {
    dim3 g(s.nblk), b(kBlock);
    if (s.pot == 0) {
        if (kick)
            hipLaunchKernelGGL((k_vertex_lj<PREC, true, false>), g, b, 0, st, s);
        else if (energy)
            hipLaunchKernelGGL((k_vertex_lj<PREC, false, true>), g, b, 0, st, s);
        else
            hipLaunchKernelGGL((k_vertex_lj<PREC, false, false>), g, b, 0, st, s);
    } else {
        if (kick)
            hipLaunchKernelGGL((k_vertex_patchy<PREC, true, false>), g, b, 0, st, s);
        else if (energy)
            hipLaunchKernelGGL((k_vertex_patchy<PREC, false, true>), g, b, 0, st, s);
        else
            hipLaunchKernelGGL((k_vertex_patchy<PREC, false, false>), g, b, 0, st, s);
    }
}

template <int PREC>
static void edge_dispatch(const Sys& s, int grid, hipStream_t st) {
    dim3 g(grid), b(kBlock);
    if (s.pot == 0)
        hipLaunchKernelGGL((k_edge<0, PREC>), g, b, 0, st, s);
    else
        hipLaunchKernelGGL((k_edge<1, PREC>), g, b, 0, st, s);
}

hipError_t launch_forces(const Sys& s, int mode, int prec, bool kick, hipStream_t st, int edge_grid) {
    if (mode == 0) {
        if (prec == 0) vertex_dispatch<0>(s, kick, false, st);
        else if (prec == 1) vertex_dispatch<1>(s, kick, false, st);
        else vertex_dispatch<2>(s, kick, false, st);
    } else {
        if (!kick) hipLaunchKernelGGL(k_zero_forces, grid_n(s.n), dim3(kBlock), 0, st, s);
        if (prec == 0) edge_dispatch<0>(s, edge_grid, st);
        else edge_dispatch<1>(s, edge_grid, st);  // FP32 pair maths, FP64 atomics
        if (kick) {
            if (s.pot == 0) hipLaunchKernelGGL(k_kick<0>, grid_n(s.n), dim3(kBlock), 0, st, s);
            else hipLaunchKernelGGL(k_kick<1>, grid_n(s.n), dim3(kBlock), 0, st, s);
        } else {
            hipLaunchKernelGGL(k_clear_rebuild, dim3(1), dim3(1), 0, st, s.ctrl);
        }
    }
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

}  // namespace md
