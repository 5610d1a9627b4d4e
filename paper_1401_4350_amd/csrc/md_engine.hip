// Host engine behind the C ABI of include/md.h: parameter validation, carving
// of the caller's two device buffers, call ordering, and the per-step launch
// sequence.  No device memory is allocated here; all work goes on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "md.h"
#include "md_internal.h"

namespace {

constexpr uint64_t kAlign = 256;
constexpr long long kSlack = 64;  // spare half-list entries
#ifndef MD_LDS_MARGIN
#define MD_LDS_MARGIN 1.45
#endif
// LDS region capacity of a tile relative to the expected region size
constexpr double kLdsMargin = MD_LDS_MARGIN;

struct Layout {
    uint64_t state_bytes = 0, ws_bytes = 0;
    // state offsets
    uint64_t pos, vel, frc, quat, angm, trq, id;
    // workspace offsets
    uint64_t pos_alt, xbuild, tpos, tposf, tvel, tquat, tangm, tid, cell, rank, ccount, cstart, order, nbr,
        ncount, hcount, hstart, hj, hr, rep, chunk_row, bsum, tmax, sync, ef, eidx, cell_rank, epart, wpart, kpart, fpl, red, ctrl, tile_seg,
        tile_nseg, tile_chunk, tile_nchunk, tile_row0;
    int nc = 0, ncell = 0, nblk = 0, ntiles = 0, lds_cap = 0, fps = 0;
    long long max_half = 0;
};

uint64_t take(uint64_t& cur, uint64_t bytes) {
    uint64_t off = cur;
    cur += (bytes + kAlign - 1) / kAlign * kAlign;
    return off;
}

md_status validate(const md_params* p) {
    if (!p) return MD_ERR_INVALID_ARG;
    auto fin = [](double v) { return std::isfinite(v); };
    if (p->n < 2 || p->n > (1 << 24) || p->max_neighbors < 1) return MD_ERR_INVALID_ARG;
    if (p->pot != MD_POT_LJ && p->pot != MD_POT_PATCHY) return MD_ERR_INVALID_ARG;
    if (p->prec < MD_PREC_FP64 || p->prec > MD_PREC_FP32_KAHAN) return MD_ERR_INVALID_ARG;
    if (!fin(p->box) || !(p->box > 0)) return MD_ERR_INVALID_ARG;
    if (!fin(p->rcut) || !(p->rcut > 0)) return MD_ERR_INVALID_ARG;
    if (!fin(p->skin) || !(p->skin >= 0)) return MD_ERR_INVALID_ARG;
    if (!fin(p->dt) || !(p->dt > 0)) return MD_ERR_INVALID_ARG;
    if (!fin(p->mass) || !(p->mass > 0)) return MD_ERR_INVALID_ARG;
    if (!fin(p->eps) || !(p->eps >= 0) || !fin(p->sigma) || !(p->sigma > 0))
        return MD_ERR_INVALID_ARG;
    if (p->pot == MD_POT_PATCHY) {
        if (!fin(p->patch_w) || !(p->patch_w > 0) || !fin(p->inertia) || !(p->inertia > 0) ||
            !fin(p->patch_delta) || !(p->patch_delta >= 0) || !fin(p->eps_p) ||
            !fin(p->patch_rcut))
            return MD_ERR_INVALID_ARG;
    }
    if (p->newton_m < 0 || p->newton_m > 64 || (p->edge_store != 0 && p->edge_store != 1))
        return MD_ERR_INVALID_ARG;
    if (p->cell_order < MD_CELLS_ROW_MAJOR || p->cell_order > MD_CELLS_HILBERT)
        return MD_ERR_INVALID_ARG;
    if (p->patch_model != MD_PATCH_TETRA &&
        (p->pot != MD_POT_PATCHY || p->patch_model != MD_PATCH_POLAR2))
        return MD_ERR_INVALID_ARG;
    // edge indices of the deterministic edge mode are 31-bit
    if (p->edge_store && (long long)p->n * p->max_neighbors / 2 + 4096 >= (long long)INT_MAX)
        return MD_ERR_INVALID_ARG;
    double rv = p->rcut + p->skin;
    if (!(p->box > 2.0 * rv)) return MD_ERR_BOX_TOO_SMALL;
    // 32-bit slot and half-list indices
    if ((long long)p->n * p->max_neighbors / 2 + kSlack > 2000000000LL)
        return MD_ERR_INVALID_ARG;
    return MD_OK;
}

}  // namespace

namespace {

// Curve index of cell (x, y, z) in a 2^b cube.  Morton: the bits of x, y, z
// interleaved (x lowest).  Hilbert: Skilling's transposition (Programming the
// Hilbert curve, AIP Conf. Proc. 707, 2004): undo the excess work of the
// recursive reflections and exchanges from the top bit down, Gray-encode
// across the axes, then interleave the transposed bits (first axis highest).
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z, int b) {
    uint64_t h = 0;
    for (int k = 0; k < b; k++)
        h |= (uint64_t)((x >> k) & 1) << (3 * k) | (uint64_t)((y >> k) & 1) << (3 * k + 1) |
             (uint64_t)((z >> k) & 1) << (3 * k + 2);
    return h;
}

uint64_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int b) {
    uint32_t X[3] = {x, y, z};
    if (b > 0) {
        const uint32_t m = 1u << (b - 1);
        for (uint32_t q = m; q > 1; q >>= 1) {
            const uint32_t p = q - 1;
            for (int i = 0; i < 3; i++) {
                if (X[i] & q) {
                    X[0] ^= p;  // invert the low bits of the first axis
                } else {        // exchange the low bits of the first axis and axis i
                    const uint32_t t = (X[0] ^ X[i]) & p;
                    X[0] ^= t;
                    X[i] ^= t;
                }
            }
        }
        for (int i = 1; i < 3; i++) X[i] ^= X[i - 1];  // Gray encode
        uint32_t t = 0;
        for (uint32_t q = m; q > 1; q >>= 1)
            if (X[2] & q) t ^= q - 1;
        for (int i = 0; i < 3; i++) X[i] ^= t;
    }
    uint64_t h = 0;
    for (int k = b - 1; k >= 0; k--)
        for (int i = 0; i < 3; i++) h = h << 1 | ((X[i] >> k) & 1);
    return h;
}

void cell_ranks(int nc, int order, int* rank) {
    const int nn = nc * nc * nc;
    if (order == MD_CELLS_ROW_MAJOR || order == MD_CELLS_ROW_MAJOR_GATHER) {
        for (int c = 0; c < nn; c++) rank[c] = c;
        return;
    }
    int b = 0;
    while ((1 << b) < nc) b++;
    std::vector<std::pair<uint64_t, int>> key(nn);
    for (int z = 0; z < nc; z++)
        for (int y = 0; y < nc; y++)
            for (int x = 0; x < nc; x++) {
                const int c = (z * nc + y) * nc + x;
                key[c] = {order == MD_CELLS_MORTON ? morton3(x, y, z, b) : hilbert3(x, y, z, b), c};
            }
    std::sort(key.begin(), key.end());
    for (int r = 0; r < nn; r++) rank[key[r].second] = r;
}

// Band of the FP32 list test around r_v^2.  A record is rounded to FP32 from
// [0, L), x_i minus an image shift from [-L, 2L), and their difference once
// more, so a component of the FP32 separation is off by at most
// delta = u (3L + r) (u = 2^-24, r the separation); the FP32 value of
// r^2 - lo (three fused multiply-adds) then differs from the exact one by at
// most 2 sqrt(3) r delta + 3 delta^2 + 3u max(r^2, lo).  With r <= 2 r_v that
// is E; below lo = r_v^2 - 2E and from lo + band >= r_v^2 + 2E on (both
// rounded outwards) the FP32 result decides as the exact one does.
void list_test_band(double box, double rv, float* lo, float* band) {
    const double u = std::ldexp(1.0, -24), r = 2.0 * rv;
    const double delta = u * (3.0 * box + r);
    const double e = 2.0 * std::sqrt(3.0) * r * delta + 3.0 * delta * delta + 3.0 * u * r * r;
    const double rv2 = rv * rv;
    *lo = std::nextafter((float)(rv2 - 2.0 * e), 0.0f);
    *band = std::nextafter((float)(rv2 + 2.0 * e - (double)*lo), INFINITY);
}

// Rows of four 32-bit entries per particle in the tiled full list: room for
// max_neighbors entries, and at least two rows (16 entries of 16 bits), the
// padding a staged tile's lists get.
uint64_t list_rows(int32_t max_neighbors) { return std::max<uint64_t>((max_neighbors + 3) / 4, 2); }

Layout layout(const md_params& p) {
    Layout L;
    uint64_t n = (uint64_t)p.n;
    double rv = p.rcut + p.skin;
    int nc = (int)std::floor(p.box / (rv * (1.0 + 1e-10)));
    nc = std::max(nc, 1);
    while ((long long)nc * nc * nc > (1LL << 26)) nc--;
    L.nc = nc;
    L.ncell = nc * nc * nc;
    L.nblk = (int)((n + md::kBlock - 1) / md::kBlock);
    L.max_half = (long long)n * p.max_neighbors / 2 + kSlack;
    L.ntiles = (int)((n + md::kTile - 1) / md::kTile);
    {
        // LDS region of a tile: the 3 x 3 rows of cells around its home cells,
        // about 9 (H + 2) cells of m particles for H home cells, with a margin;
        // tiles that still do not fit use global gathers.
        double m = (double)n / L.ncell;
        double h = md::kTile / std::max(m, 1e-3) + 1.0;
        double expect = 9.0 * (h + 2.0) * m;
        int cap = (int)std::ceil(kLdsMargin * expect / 64.0) * 64;
        L.lds_cap = std::min(std::max(cap, 512), md::kLdsCapMax);
    }
    bool patchy = p.pot == MD_POT_PATCHY;
    uint64_t d4 = 32 * n;
    uint64_t cur = 0;
    L.pos = take(cur, d4);
    L.vel = take(cur, d4);
    L.frc = take(cur, d4);
    L.quat = take(cur, patchy ? d4 : 0);
    L.angm = take(cur, patchy ? d4 : 0);
    L.trq = take(cur, patchy ? d4 : 0);
    L.id = take(cur, 4 * n);
    L.state_bytes = cur;
    cur = 0;
    L.ctrl = take(cur, sizeof(md::Ctrl));
    L.pos_alt = take(cur, d4);
    L.xbuild = take(cur, d4);
    L.tpos = take(cur, d4);
    L.tposf = take(cur, 16 * (n + md::kRunPad));
    L.tvel = take(cur, d4);
    L.tquat = take(cur, patchy ? d4 : 0);
    L.tangm = take(cur, patchy ? d4 : 0);
    L.tid = take(cur, 4 * n);
    L.cell = take(cur, 4 * n);
    L.rank = take(cur, 4 * n);
    L.ccount = take(cur, 4 * (uint64_t)L.ncell);
    L.cstart = take(cur, 4 * ((uint64_t)L.ncell + 1));
    L.order = take(cur, 4 * n);
    L.nbr = take(cur, 4 * ((uint64_t)L.ntiles * list_rows(p.max_neighbors) + md::kListPadRows) *
                          md::kTile * 4);
    L.ncount = take(cur, 4 * n);
    L.hcount = take(cur, 4 * n);
    L.hstart = take(cur, 4 * (n + 1));
    L.hj = take(cur, 4 * (uint64_t)L.max_half);
    // packed words of the edge passes (row in the tile, region index of the
    // partner), four spare (the LJ pass reads them four at a time)
    L.hr = take(cur, 4 * ((uint64_t)L.max_half + 4));
    // Newton mode replicas: m force arrays (and for patchy m torque arrays)
    L.rep = take(cur, (p.pot == MD_POT_LJ ? 32 : 64) * n * (uint64_t)p.newton_m);
    L.chunk_row = take(cur, 4 * ((uint64_t)L.max_half / md::kWave + 2));
    L.bsum = take(cur, 4 * (uint64_t)std::max(L.nblk, L.ntiles));  // per-tile half totals
    L.tmax = take(cur, 4 * (uint64_t)L.ntiles);
    L.cell_rank = take(cur, p.cell_order >= MD_CELLS_MORTON ? 4 * (uint64_t)L.ncell : 0);
    // deterministic edge mode: per-edge results (F, and tau_i, tau_j for
    // patchy) and an edge index per full-list entry
    const uint64_t nrec = p.pot == MD_POT_LJ ? 1 : 3;
    L.ef = take(cur, p.edge_store ? 32 * nrec * (uint64_t)L.max_half : 0);
    L.eidx = take(cur, p.edge_store ? 4 * (uint64_t)L.ntiles * list_rows(p.max_neighbors) * md::kTile * 4 : 0);
    L.sync = take(cur, 4 * (uint64_t)md::kSyncUses * md::kSyncInts);
    L.tile_seg = take(cur, 16 * (uint64_t)L.ntiles * md::kSegMax);
    L.tile_nseg = take(cur, 4 * (uint64_t)L.ntiles);
    L.tile_chunk = take(cur, 16 * (uint64_t)L.ntiles * md::kChunkMax);
    L.tile_nchunk = take(cur, 4 * (uint64_t)L.ntiles);
    L.tile_row0 = take(cur, 4 * (uint64_t)L.ntiles);
    L.epart = take(cur, 8 * n);
    L.wpart = take(cur, 8 * n);
    L.kpart = take(cur, 8 * n);
    // LJ edge pass: force planes (x, y, z of every slot in arrays of their
    // own), each plane padded to a multiple of 32 doubles
    L.fps = (int)((n + 31) / 32 * 32);
    L.fpl = take(cur, p.pot == MD_POT_LJ ? 24 * (uint64_t)L.fps : 0);
    L.red = take(cur, 8 * (3 * (uint64_t)md::kRedBlocks + 3));
    L.ws_bytes = cur;
    return L;
}

const char* status_text(int s) {
    switch (s) {
        case MD_OK: return "ok";
        case MD_ERR_INVALID_ARG: return "invalid argument";
        case MD_ERR_BUFFER_TOO_SMALL: return "buffer too small or misaligned";
        case MD_ERR_HIP: return "HIP runtime error";
        case MD_ERR_NEIGHBOR_OVERFLOW: return "Verlet list overflow (raise max_neighbors)";
        case MD_ERR_BOX_TOO_SMALL: return "box must exceed 2 (rcut + skin)";
        case MD_ERR_NONFINITE: return "non-finite force or position";
        case MD_ERR_STATE: return "call out of order";
        default: return "unknown status";
    }
}

}  // namespace

struct md_system {
    md_params p;
    Layout lay;
    md::Sys sys;
    hipStream_t stream;
    bool state_set = false;
    bool cells_pending = false;
    bool lists_valid = false;
    bool forces_valid = false;
    long long steps = 0;
    int edge_grid = 1;
    md_batch* batch = nullptr;  // set while admitted to a batch
    int batch_slot = -1;
    std::string err;
    // md_step phase timing (md_profile_enable)
    bool profiling = false;
    std::vector<hipEvent_t> events;  // 4 per step of the current md_step call
    md_profile_t prof{};
    // fused vertex steps: launch ids, the host-mapped word in which every
    // launch that runs leaves its id, and one event per batch in flight
    int next_id = 2;
    int* run_host = nullptr;
    int* run_dev = nullptr;
    hipEvent_t fev[2] = {nullptr, nullptr};

    ~md_system() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipEvent_t e : fev)
            if (e) (void)hipEventDestroy(e);
        if (run_host) (void)hipHostFree(run_host);
    }
    // A pinned, host-mapped word and two events, made on the first fused step.
    hipError_t fused_setup() {
        if (run_host) return hipSuccess;
        void* h = nullptr;
        hipError_t r = hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent);
        if (r != hipSuccess) return r;
        run_host = static_cast<int*>(h);
        *run_host = 0;
        void* d = nullptr;
        r = hipHostGetDevicePointer(&d, h, 0);
        if (r != hipSuccess) return r;
        run_dev = static_cast<int*>(d);
        for (hipEvent_t& e : fev) {
            r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (r != hipSuccess) return r;
        }
        sys.host_run = run_dev;
        return hipSuccess;
    }
    // Ids for the next n fused launches, consecutive from the returned one
    // (they restart, with the request slots cleared, long before they could
    // overflow).
    hipError_t reserve_ids(int n) {
        if (next_id + n < (1 << 30)) return hipSuccess;
        char* req = reinterpret_cast<char*>(sys.ctrl) + offsetof(md::Ctrl, req);
        hipError_t r = hipMemsetAsync(req, 0, sizeof(md::Ctrl::req), stream);
        next_id = 2;
        return r;
    }
    hipError_t ensure_events(size_t count) {
        while (events.size() < count) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            events.push_back(e);
        }
        return hipSuccess;
    }

    md_status fail(md_status st, const std::string& msg) {
        err = msg;
        return st;
    }
    md_status admitted() {
        return fail(MD_ERR_STATE, "the system is admitted to a batch; md_batch_retire it first");
    }
    md_status hip(hipError_t e, const char* where) {
        if (e == hipSuccess) return MD_OK;
        err = std::string(where) + ": " + hipGetErrorString(e);
        return MD_ERR_HIP;
    }
    // Waits for the stream and turns sticky device flags into a status.
    md_status sync_check() {
        md_status st = hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
        if (st != MD_OK) return st;
        md::Ctrl c;
        st = hip(hipMemcpy(&c, sys.ctrl, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy(ctrl)");
        if (st != MD_OK) return st;
        if (c.overflow & 2)
            return fail(MD_ERR_STATE, "internal: a tile region misses a neighbour cell");
        if (c.overflow)
            return fail(MD_ERR_NEIGHBOR_OVERFLOW,
                        "a Verlet list exceeded max_neighbors=" + std::to_string(p.max_neighbors) +
                            " (longest " + std::to_string(c.max_count) + ")");
        if (c.nonfinite) return fail(MD_ERR_NONFINITE, "non-finite force");
        return MD_OK;
    }
};

extern "C" {

md_status md_cell_order_ranks(int32_t nc, int32_t order, int32_t* rank) {
    if (!rank || nc < 1 || nc > 1024 || order < MD_CELLS_ROW_MAJOR || order > MD_CELLS_HILBERT)
        return MD_ERR_INVALID_ARG;
    cell_ranks(nc, order, rank);
    return MD_OK;
}

md_status md_query_sizes(const md_params* p, md_sizes* out) {
    if (!out) return MD_ERR_INVALID_ARG;
    md_status st = validate(p);
    if (st != MD_OK) return st;
    Layout L = layout(*p);
    out->state_bytes = L.state_bytes;
    out->workspace_bytes = L.ws_bytes;
    out->alignment = kAlign;
    return MD_OK;
}

}  // extern "C"

namespace {

// The kernels' descriptor of a system whose state and workspace start at
// d_state and d_workspace (carved as `layout` says); *edge_grid gets the
// block count of the edge pass.
void fill_sys(const md_params* p, const Layout& L, void* d_state, void* d_workspace, md::Sys& y,
              int* edge_grid) {
    std::memset(&y, 0, sizeof y);
    char* S = (char*)d_state;
    char* W = (char*)d_workspace;
    bool patchy = p->pot == MD_POT_PATCHY;
    y.n = p->n;
    y.nc = L.nc;
    y.ncell = L.ncell;
    y.cap = p->max_neighbors;
    y.mcap = (int)list_rows(p->max_neighbors);
    y.pot = p->pot;
    y.nblk = L.nblk;
    y.max_half = L.max_half;
    y.box = p->box;
    y.inv_box = 1.0 / p->box;
    y.cell_inv = L.nc / p->box;
    double rv = p->rcut + p->skin;
    y.rv2 = rv * rv;
    list_test_band(p->box, rv, &y.rv2_lo, &y.rv2_band);
    y.rc2 = p->rcut * p->rcut;
    y.disp2 = 0.25 * p->skin * p->skin;
    y.dt = p->dt;
    y.hdt = 0.5 * p->dt;
    y.inv_mass = 1.0 / p->mass;
    y.inv_inertia = patchy ? 1.0 / p->inertia : 0.0;
    md::set_potential(y, p->eps, p->sigma, p->rcut, p->eps_p, patchy ? p->patch_w : 1.0,
                      p->patch_delta, p->patch_rcut, p->patch_model);
    y.pos = (double4*)(S + L.pos);
    y.vel = (double4*)(S + L.vel);
    y.frc = (double4*)(S + L.frc);
    y.quat = patchy ? (double4*)(S + L.quat) : nullptr;
    y.angm = patchy ? (double4*)(S + L.angm) : nullptr;
    y.trq = patchy ? (double4*)(S + L.trq) : nullptr;
    y.id = (int*)(S + L.id);
    y.ctrl = (md::Ctrl*)(W + L.ctrl);
    y.pos_alt = (double4*)(W + L.pos_alt);
    y.xbuild = (double4*)(W + L.xbuild);
    y.tpos = (double4*)(W + L.tpos);
    y.tposf = (float4*)(W + L.tposf);
    y.tvel = (double4*)(W + L.tvel);
    y.tquat = patchy ? (double4*)(W + L.tquat) : nullptr;
    y.tangm = patchy ? (double4*)(W + L.tangm) : nullptr;
    y.tid = (int*)(W + L.tid);
    y.cell = (int*)(W + L.cell);
    y.rank = (int*)(W + L.rank);
    y.ccount = (int*)(W + L.ccount);
    y.cstart = (int*)(W + L.cstart);
    y.order = (int*)(W + L.order);
    y.nbr = (int*)(W + L.nbr);
    y.ncount = (int*)(W + L.ncount);
    y.hcount = (int*)(W + L.hcount);
    y.hstart = (int*)(W + L.hstart);
    y.hj = (int*)(W + L.hj);
    y.hr = (unsigned*)(W + L.hr);
    y.rep = (double4*)(W + L.rep);
    y.nrep = p->newton_m;
    y.chunk_row = (int*)(W + L.chunk_row);
    y.bsum = (int*)(W + L.bsum);
    y.tmax = (int*)(W + L.tmax);
    y.estore = p->edge_store;
    y.cell_order = p->cell_order;
    y.cell_rank = p->cell_order >= MD_CELLS_MORTON ? (const int*)(W + L.cell_rank) : nullptr;
    y.ef = p->edge_store ? (double4*)(W + L.ef) : nullptr;
    y.eidx = p->edge_store ? (int*)(W + L.eidx) : nullptr;
    y.sync = (int*)(W + L.sync);
    y.ntiles = L.ntiles;
    y.lds_cap = L.lds_cap;
    y.tile_seg = (int4*)(W + L.tile_seg);
    y.tile_nseg = (int*)(W + L.tile_nseg);
    y.tile_chunk = (int4*)(W + L.tile_chunk);
    y.tile_nchunk = (int*)(W + L.tile_nchunk);
    y.tile_row0 = (int*)(W + L.tile_row0);
    y.epart = (double*)(W + L.epart);
    y.wpart = (double*)(W + L.wpart);
    y.kpart = (double*)(W + L.kpart);
    y.fpl = (double*)(W + L.fpl);
    y.fps = L.fps;
    y.red = (double*)(W + L.red);

    long long waves = (L.max_half + md::kWave - 1) / md::kWave;
    long long blocks = (waves + 3) / 4;
    *edge_grid = (int)std::max(1LL, std::min(blocks, 4096LL));
    y.prec = p->prec;
}

// md_create with the workspace given (validated by the caller).
md_status create_system(const md_params* p, const Layout& L, void* d_state, void* d_workspace,
                        void* hip_stream, md_system** out) {
    md_status st = MD_OK;
    md_system* s = new md_system();
    s->p = *p;
    s->lay = L;
    s->stream = (hipStream_t)hip_stream;
    md::Sys& y = s->sys;
    fill_sys(p, L, d_state, d_workspace, y, &s->edge_grid);
    bool patchy = p->pot == MD_POT_PATCHY;

    // One-time clears at creation (never inside a captured step).
    st = s->hip(hipMemsetAsync(y.ccount, 0, 4 * (size_t)L.ncell, s->stream), "clear cell counts");
    if (st == MD_OK) st = s->hip(hipMemsetAsync(d_state, 0, L.state_bytes, s->stream), "clear state");
    if (st == MD_OK && y.nrep > 0)  // replicas start at zero; the combining pass re-zeroes them
        st = s->hip(hipMemsetAsync(y.rep, 0, (patchy ? 64 : 32) * (size_t)p->n * y.nrep, s->stream),
                    "clear replicas");
    std::vector<int> ranks;  // cell order table, copied before the stream is drained
    if (st == MD_OK && y.cell_rank) {
        ranks.resize(L.ncell);
        cell_ranks(L.nc, p->cell_order, ranks.data());
        st = s->hip(hipMemcpyAsync((void*)y.cell_rank, ranks.data(), 4 * (size_t)L.ncell,
                                   hipMemcpyHostToDevice, s->stream),
                    "cell order");
    }
    if (st == MD_OK) st = s->hip(md::launch_clear_ctrl(y, s->stream), "clear control");
    if (st == MD_OK) st = s->hip(hipStreamSynchronize(s->stream), "create sync");
    if (st != MD_OK) {
        delete s;
        return st;
    }
    *out = s;
    return MD_OK;
}

}  // namespace

extern "C" {

md_status md_create(const md_params* p, void* d_state, uint64_t state_bytes, void* d_workspace,
                    uint64_t workspace_bytes, void* hip_stream, md_system** out) {
    if (!out) return MD_ERR_INVALID_ARG;
    *out = nullptr;
    md_status st = validate(p);
    if (st != MD_OK) return st;
    if (!d_state || !d_workspace) return MD_ERR_INVALID_ARG;
    Layout L = layout(*p);
    if (state_bytes < L.state_bytes || workspace_bytes < L.ws_bytes) return MD_ERR_BUFFER_TOO_SMALL;
    if ((uintptr_t)d_state % kAlign || (uintptr_t)d_workspace % kAlign)
        return MD_ERR_BUFFER_TOO_SMALL;
    return create_system(p, L, d_state, d_workspace, hip_stream, out);
}


}  // extern "C"

// ---------------------------------------------------------------------------
// md_forces_static: the forces of md_forces for coordinates already on the
// device, with no caller workspace.  State and workspace live in `scratch`,
// a file-scope device array that every GPU the library runs on holds once
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address reaches the kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MD_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
md_status static_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MD_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MD_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MD_OK;
}

}  // namespace

extern "C" {

md_status md_forces_static(const md_params* p, const double* d_x, const double* d_q,
                           double* d_f, double* d_torque, int32_t mode, int32_t* d_status,
                           void* hip_stream) {
    md_status st = validate(p);
    if (st != MD_OK) return st;
    // state and workspace back to back, as md_query_sizes reports them
    const Layout L = layout(*p);
    if (L.state_bytes + L.ws_bytes > MD_STATIC_SCRATCH_BYTES) return MD_ERR_BUFFER_TOO_SMALL;
    const bool patchy = p->pot == MD_POT_PATCHY;
    if (!d_x || !d_f || (patchy && (!d_q || !d_torque))) return MD_ERR_INVALID_ARG;
    if (mode != MD_MODE_VERTEX && mode != MD_MODE_EDGE && mode != MD_MODE_NEWTON &&
        mode != MD_MODE_EDGE_DET)
        return MD_ERR_INVALID_ARG;
    if (mode == MD_MODE_EDGE_DET && !p->edge_store) return MD_ERR_INVALID_ARG;
    // the curve orders need a host-built rank table uploaded per call
    if (p->cell_order != MD_CELLS_ROW_MAJOR && p->cell_order != MD_CELLS_ROW_MAJOR_GATHER)
        return MD_ERR_INVALID_ARG;
    void* base = nullptr;
    st = static_scratch(&base);
    if (st != MD_OK) return st;
    md::Sys y;
    int edge_grid = 1;
    fill_sys(p, L, base, (char*)base + L.state_bytes, y, &edge_grid);
    hipStream_t s = (hipStream_t)hip_stream;
    // The array keeps the previous call's contents, possibly of another
    // layout: clear what the passes expect at zero (cell counts, completion
    // counters and the control block, Newton replicas) with fill kernels.
    hipError_t e = md::launch_fill_zero(y.ccount, L.ncell, s);
    if (e == hipSuccess && y.nrep > 0)
        e = md::launch_fill_zero((int*)y.rep, (long long)(patchy ? 16 : 8) * p->n * y.nrep, s);
    if (e == hipSuccess) e = md::launch_clear_ctrl(y, s);
    if (e == hipSuccess) e = md::launch_load_records(y, d_x, patchy ? d_q : nullptr, s);
    // md_build_cells, md_build_neighbors, md_forces
    if (e == hipSuccess) e = md::launch_set_rebuild(y, s);
    if (e == hipSuccess) e = md::launch_rebuild(y, s, true, false);
    if (e == hipSuccess) e = md::launch_rebuild(y, s, false, true);
    if (e == hipSuccess) e = md::launch_clear_rebuild(y, s);
    if (e == hipSuccess) e = md::launch_forces(y, mode, p->prec, false, s, edge_grid);
    if (e == hipSuccess) e = md::launch_store_results(y, d_f, patchy ? d_torque : nullptr, s);
    if (e == hipSuccess && d_status)
        e = md::launch_status(y, d_status, MD_ERR_NEIGHBOR_OVERFLOW, MD_ERR_NONFINITE, s);
    return e == hipSuccess ? MD_OK : MD_ERR_HIP;
}


md_status md_set_state(md_system* s, const double* x, const double* v, const double* q,
                       const double* angmom) {
    if (!s || !x || !v) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    bool patchy = s->p.pot == MD_POT_PATCHY;
    if (patchy && (!q || !angmom)) return s->fail(MD_ERR_INVALID_ARG, "patchy needs q and angmom");
    int n = s->p.n;
    double L = s->p.box;
    std::vector<double4> hp(n), hv(n), hq, hl;
    std::vector<int> hid(n);
    for (int i = 0; i < n; i++) {
        double c[3];
        for (int k = 0; k < 3; k++) {
            double y = x[3 * i + k];
            if (!std::isfinite(y) || !std::isfinite(v[3 * i + k]))
                return s->fail(MD_ERR_NONFINITE, "non-finite input state");
            y -= L * std::floor(y / L);
            if (y >= L) y -= L;
            if (y < 0) y += L;
            c[k] = y;
        }
        hp[i] = make_double4(c[0], c[1], c[2], 0.0);
        hv[i] = make_double4(v[3 * i], v[3 * i + 1], v[3 * i + 2], 0.0);
        hid[i] = i;
    }
    if (patchy) {
        hq.resize(n);
        hl.resize(n);
        for (int i = 0; i < n; i++) {
            const double* a = q + 4 * i;
            double nn = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
            if (!(nn > 0) || !std::isfinite(nn))
                return s->fail(MD_ERR_INVALID_ARG, "quaternion must be non-zero");
            hq[i] = make_double4(a[0] / nn, a[1] / nn, a[2] / nn, a[3] / nn);
            hl[i] = make_double4(angmom[3 * i], angmom[3 * i + 1], angmom[3 * i + 2], 0.0);
        }
    }
    md::Sys& y = s->sys;
    hipStream_t st = s->stream;
    size_t b4 = sizeof(double4) * (size_t)n;
    md_status r = s->hip(hipMemcpyAsync(y.pos, hp.data(), b4, hipMemcpyHostToDevice, st), "upload x");
    if (r == MD_OK) r = s->hip(hipMemcpyAsync(y.vel, hv.data(), b4, hipMemcpyHostToDevice, st), "upload v");
    if (r == MD_OK) r = s->hip(hipMemcpyAsync(y.id, hid.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st), "upload id");
    if (r == MD_OK) r = s->hip(hipMemsetAsync(y.frc, 0, b4, st), "clear F");
    if (patchy) {
        if (r == MD_OK) r = s->hip(hipMemcpyAsync(y.quat, hq.data(), b4, hipMemcpyHostToDevice, st), "upload q");
        if (r == MD_OK) r = s->hip(hipMemcpyAsync(y.angm, hl.data(), b4, hipMemcpyHostToDevice, st), "upload L");
        if (r == MD_OK) r = s->hip(hipMemsetAsync(y.trq, 0, b4, st), "clear tau");
    }
    if (r == MD_OK) r = s->hip(md::launch_clear_ctrl(y, st), "clear control");
    if (r == MD_OK) r = s->hip(hipStreamSynchronize(st), "set_state sync");
    if (r != MD_OK) return r;
    s->state_set = true;
    s->cells_pending = false;
    s->lists_valid = false;
    s->forces_valid = false;
    s->err.clear();
    return MD_OK;
}

md_status md_build_cells(md_system* s) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (!s->state_set) return s->fail(MD_ERR_STATE, "md_set_state first");
    md_status r = s->hip(md::launch_set_rebuild(s->sys, s->stream), "set rebuild");
    if (r == MD_OK) r = s->hip(md::launch_rebuild(s->sys, s->stream, true, false), "cell sort");
    if (r != MD_OK) return r;
    s->cells_pending = true;
    s->lists_valid = false;
    s->forces_valid = false;
    return MD_OK;
}

md_status md_build_neighbors(md_system* s) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (!s->cells_pending) return s->fail(MD_ERR_STATE, "md_build_cells first");
    md_status r = s->hip(md::launch_rebuild(s->sys, s->stream, false, true), "list build");
    if (r == MD_OK) r = s->hip(md::launch_clear_rebuild(s->sys, s->stream), "clear rebuild");
    if (r != MD_OK) return r;
    s->cells_pending = false;
    s->lists_valid = true;
    s->forces_valid = false;
    return MD_OK;
}

static md_status check_mode(md_system* s, int32_t mode) {
    if (mode != MD_MODE_VERTEX && mode != MD_MODE_EDGE && mode != MD_MODE_NEWTON &&
        mode != MD_MODE_EDGE_DET)
        return s->fail(MD_ERR_INVALID_ARG, "mode");
    if (mode == MD_MODE_EDGE_DET && !s->p.edge_store)
        return s->fail(MD_ERR_INVALID_ARG, "the deterministic edge mode needs edge_store = 1 at md_create");
    return MD_OK;
}

md_status md_forces(md_system* s, int32_t mode) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    md_status r = check_mode(s, mode);
    if (r != MD_OK) return r;
    if (!s->lists_valid) return s->fail(MD_ERR_STATE, "md_build_neighbors first");
    r = s->hip(md::launch_forces(s->sys, mode, s->p.prec, false, s->stream, s->edge_grid),
                         "forces");
    if (r != MD_OK) return r;
    s->forces_valid = true;
    return MD_OK;
}

// Fused vertex LJ steps without the rebuild test chain in every step.  Each
// fused launch (forces, closing and next half kick, drift) checks at its start
// whether the drift of the launch before asked for a list rebuild, and if so
// does nothing but pass the request on (Ctrl::req).  The host enqueues the
// launches in batches of kFusedBatch, two batches ahead, and after each batch
// reads the id of the last launch that ran (a host-mapped word): if a batch
// stopped early, it waits for the rest, runs the rebuild chain on the
// positions of the last launch that ran and resumes from there.  The four
// launches of the chain (each of which returns at once when no rebuild is
// due) then run only at rebuilds instead of in every step.  Same arithmetic,
// same rebuild steps as the per-step sequence.
constexpr int kFusedBatch = 4;

static md_status step_fused(md_system* s, int nsteps) {
    hipStream_t st = s->stream;
    md::Sys y = s->sys;
    double4* const pa = y.pos;
    double4* const pb = y.pos_alt;
    auto parity = [&](int ran) {  // the positions after `ran` fused launches
        y.pos = (ran & 1) ? pb : pa;
        y.pos_alt = (ran & 1) ? pa : pb;
    };
    auto fail = [&](hipError_t e, const char* where) {
        s->sys = y;
        return s->hip(e, where);
    };
    // step 0: half kick and drift, then the rebuild test chain
    hipError_t e = md::launch_kick_drift(y, false, st);
    if (e == hipSuccess) e = md::launch_rebuild(y, st, true, true);
    if (e != hipSuccess) return fail(e, "step launch");
    const int nfused = nsteps - 1;  // fused launches that must run
    int done = 0;                   // of which known to have run
    int issued = 0;                 // enqueued after those, not yet confirmed
    struct Batch {
        int first, n;
    } q[2];
    int head = 0, inflight = 0;
    int stalls = 0;  // rebuilds in a row after which no launch ran
    while (done < nfused) {
        while (inflight < 2 && done + issued < nfused) {
            const int k = (head + inflight) & 1;
            const int n = std::min(kFusedBatch, nfused - done - issued);
            e = s->reserve_ids(n);
            if (e != hipSuccess) return fail(e, "fused step ids");
            q[k].first = s->next_id;
            q[k].n = n;
            for (int j = 0; j < n; j++) {
                y.launch_id = s->next_id++;
                e = md::launch_vertex_kick_drift(y, s->p.prec, st);
                if (e != hipSuccess) return fail(e, "fused step launch");
                std::swap(y.pos, y.pos_alt);
            }
            e = hipEventRecord(s->fev[k], st);
            if (e != hipSuccess) return fail(e, "fused step event");
            issued += n;
            inflight++;
        }
        e = hipEventSynchronize(s->fev[head]);
        if (e != hipSuccess) return fail(e, "fused step wait");
        const Batch b = q[head];
        head ^= 1;
        inflight--;
        const int last = *(volatile int*)s->run_host;
        const int ran = last >= b.first ? std::min(last - b.first + 1, b.n) : 0;
        done += ran;
        issued -= b.n;
        stalls = ran > 0 ? 0 : stalls + 1;
        if (stalls > 2) {  // a rebuild that does not let the next launch run: a bug, not a hang
            s->sys = y;
            return s->fail(MD_ERR_STATE, "internal: fused steps make no progress");
        }
        if (ran < b.n) {
            // a rebuild is due: every later launch does nothing, the batch
            // still in flight included, so the rebuild chain is enqueued
            // behind it at once (the stream keeps the order; waiting for
            // that batch first would leave the GPU idle while the host
            // catches up)
            if (inflight) {
                issued -= q[head].n;
                head ^= 1;
                inflight = 0;
            }
            parity(done);
            s->next_id++;  // not the successor of a launch that passed the request on
            e = md::launch_rebuild(y, st, true, true);
            if (e != hipSuccess) return fail(e, "rebuild launch");
        }
    }
    parity(done);
    // last step: the rebuild test chain, forces and the closing kick
    e = md::launch_rebuild(y, st, true, true);
    if (e == hipSuccess) e = md::launch_forces(y, MD_MODE_VERTEX, s->p.prec, true, st, s->edge_grid);
    if (e != hipSuccess) return fail(e, "step launch");
    s->sys = y;
    s->steps += nsteps;
    return s->sync_check();
}

md_status md_step(md_system* s, int32_t nsteps, int32_t mode) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (nsteps < 0) return s->fail(MD_ERR_INVALID_ARG, "nsteps");
    md_status rm = check_mode(s, mode);
    if (rm != MD_OK) return rm;
    if (!s->lists_valid) return s->fail(MD_ERR_STATE, "md_build_neighbors first");
    if (!s->forces_valid) {
        md_status r = md_forces(s, mode);
        if (r != MD_OK) return r;
    }
    // The vertex LJ pass also does the next step's half kick and drift (into
    // the second position buffer, whose role swaps with the first every
    // fused step), so after the first step one MD step is the rebuild test
    // chain and one force launch.
    const bool fuse = mode == MD_MODE_VERTEX && s->p.pot == MD_POT_LJ;
    bool prof = s->profiling;
    if (fuse) {
        md_status r = s->hip(s->fused_setup(), "fused step setup");
        if (r != MD_OK) return r;
        if (!prof && nsteps >= 2) return step_fused(s, nsteps);
    }
    md::Sys y = s->sys;
    // passes that add with atomics into the force array need it cleared first
    bool edge = mode == MD_MODE_EDGE || (mode == MD_MODE_NEWTON && s->sys.nrep == 0);
    constexpr size_t kEv = 5;  // events per profiled step
    if (prof) {
        md_status r = s->hip(s->ensure_events(kEv * (size_t)nsteps), "profile events");
        if (r != MD_OK) return r;
    }
    hipStream_t st = s->stream;
    for (int k = 0; k < nsteps; k++) {
        hipEvent_t* ev = prof ? &s->events[kEv * (size_t)k] : nullptr;
        hipError_t e = prof ? hipEventRecord(ev[0], st) : hipSuccess;
        if (e == hipSuccess && (!fuse || k == 0)) e = md::launch_kick_drift(y, edge, st);
        if (e == hipSuccess && prof) e = hipEventRecord(ev[1], st);
        if (e == hipSuccess) e = md::launch_rebuild(y, st, true, true);
        if (e == hipSuccess && prof) e = hipEventRecord(ev[2], st);
        if (fuse && k + 1 < nsteps) {
            if (e == hipSuccess) e = s->reserve_ids(1);
            y.launch_id = s->next_id++;
            if (e == hipSuccess) e = md::launch_vertex_kick_drift(y, s->p.prec, st);
            std::swap(y.pos, y.pos_alt);
            if (e == hipSuccess && prof) e = hipEventRecord(ev[3], st);
        } else if (e == hipSuccess) {
            // the closing kick of the passes without a fused one comes after
            // event 3, so the force phase times the force kernels alone
            e = md::launch_forces(y, mode, s->p.prec, true, st, s->edge_grid,
                                  prof ? ev[3] : nullptr);
        }
        if (e == hipSuccess && prof) e = hipEventRecord(ev[4], st);
        if (e != hipSuccess) {
            s->sys = y;
            return s->hip(e, "step launch");
        }
    }
    s->sys = y;
    s->steps += nsteps;
    md_status r = s->sync_check();
    if (r != MD_OK || !prof) return r;
    for (int k = 0; k < nsteps; k++) {
        hipEvent_t* ev = &s->events[kEv * (size_t)k];
        float a = 0, b = 0, c = 0, d = 0;
        hipError_t e = hipEventElapsedTime(&a, ev[0], ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[1], ev[2]);
        if (e == hipSuccess) e = hipEventElapsedTime(&c, ev[2], ev[3]);
        if (e == hipSuccess) e = hipEventElapsedTime(&d, ev[3], ev[4]);
        if (e != hipSuccess) return s->hip(e, "profile elapsed");
        s->prof.integrate_ms += a;
        s->prof.rebuild_ms += b;
        s->prof.force_ms += c;
        s->prof.kick_ms += d;
    }
    s->prof.steps += nsteps;
    return MD_OK;
}

md_status md_thermostat(md_system* s, double temperature, double prob, uint64_t seed,
                        uint64_t counter) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (!std::isfinite(temperature) || !(temperature >= 0) || !(prob >= 0) || !(prob <= 1))
        return s->fail(MD_ERR_INVALID_ARG, "thermostat needs temperature >= 0 and 0 <= prob <= 1");
    if (!s->state_set) return s->fail(MD_ERR_STATE, "md_set_state first");
    // between md_build_cells and md_build_neighbors the momenta sit in the
    // reorder buffers, which the list build copies back over the state
    if (s->cells_pending) return s->fail(MD_ERR_STATE, "md_build_neighbors first");
    const double sv = std::sqrt(temperature / s->p.mass);
    const double sl = s->p.pot == MD_POT_PATCHY ? std::sqrt(s->p.inertia * temperature) : 0.0;
    return s->hip(md::launch_thermostat(s->sys, sv, sl, prob, seed, counter, s->stream),
                  "thermostat");
}

md_status md_profile_enable(md_system* s, int32_t on) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    s->profiling = on != 0;
    s->prof = md_profile_t{};
    return MD_OK;
}

md_status md_profile_read(md_system* s, md_profile_t* out) {
    if (!s || !out) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    md_status r = s->hip(hipStreamSynchronize(s->stream), "profile sync");
    if (r != MD_OK) return r;
    *out = s->prof;
    return MD_OK;
}

md_status md_energy(md_system* s, double* e_kin, double* e_pot, double* virial) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (!s->lists_valid) return s->fail(MD_ERR_STATE, "md_build_neighbors first");
    md_status r = s->hip(md::launch_energy(s->sys, s->p.prec, s->stream), "energy");
    if (r != MD_OK) return r;
    double h[3];
    r = s->hip(hipMemcpyAsync(h, s->sys.red + 3 * md::kRedBlocks, sizeof h, hipMemcpyDeviceToHost,
                              s->stream),
               "energy download");
    if (r == MD_OK) r = s->sync_check();
    if (r != MD_OK) return r;
    if (e_kin) *e_kin = h[0];
    if (e_pot) *e_pot = h[1];
    if (virial) *virial = h[2];
    return MD_OK;
}

static md_status download_ids(md_system* s, std::vector<int>& id) {
    id.resize(s->p.n);
    return s->hip(hipMemcpyAsync(id.data(), s->sys.id, 4 * (size_t)s->p.n, hipMemcpyDeviceToHost,
                                 s->stream),
                  "download ids");
}

md_status md_particle_energies(md_system* s, double* e) {
    if (!s || !e) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (!s->lists_valid) return s->fail(MD_ERR_STATE, "md_build_neighbors first");
    int n = s->p.n;
    std::vector<double> h(n);
    std::vector<int> id;
    md_status r = s->hip(md::launch_energy(s->sys, s->p.prec, s->stream), "energy");
    if (r == MD_OK)
        r = s->hip(hipMemcpyAsync(h.data(), s->sys.epart, 8 * (size_t)n, hipMemcpyDeviceToHost,
                                  s->stream),
                   "download e");
    if (r == MD_OK) r = download_ids(s, id);
    if (r == MD_OK) r = s->sync_check();
    if (r != MD_OK) return r;
    for (int k = 0; k < n; k++) e[id[k]] = h[k];
    return MD_OK;
}

md_status md_get_state(md_system* s, double* x, double* v, double* f, double* q, double* angmom,
                       double* torque) {
    if (!s) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (!s->state_set) return s->fail(MD_ERR_STATE, "md_set_state first");
    bool patchy = s->p.pot == MD_POT_PATCHY;
    if (!patchy && (q || angmom || torque)) return s->fail(MD_ERR_INVALID_ARG, "LJ has no rotation");
    int n = s->p.n;
    std::vector<int> id;
    md_status r = download_ids(s, id);
    struct Item {
        double* dst;
        double4* src;
        int width;
    } items[6] = {{x, s->sys.pos, 3},     {v, s->sys.vel, 3},    {f, s->sys.frc, 3},
                  {q, s->sys.quat, 4},    {angmom, s->sys.angm, 3}, {torque, s->sys.trq, 3}};
    std::vector<double4> buf(n);
    if (r == MD_OK) r = s->hip(hipStreamSynchronize(s->stream), "get_state sync");
    for (auto& it : items) {
        if (r != MD_OK || !it.dst) continue;
        r = s->hip(hipMemcpy(buf.data(), it.src, sizeof(double4) * (size_t)n, hipMemcpyDeviceToHost),
                   "download state");
        if (r != MD_OK) break;
        bool is_pos = it.src == s->sys.pos;  // unwrapped between builds: wrap into [0, L)
        double L = s->p.box;
        for (int k = 0; k < n; k++) {
            double* d = it.dst + (size_t)it.width * id[k];
            d[0] = buf[k].x;
            d[1] = buf[k].y;
            d[2] = buf[k].z;
            if (it.width == 4) d[3] = buf[k].w;
            if (is_pos)
                for (int c = 0; c < 3; c++) {
                    if (d[c] >= L) d[c] -= L;
                    if (d[c] < 0) d[c] += L;
                }
        }
    }
    if (r != MD_OK) return r;
    return s->sync_check();
}

md_status md_get_pairs(md_system* s, int32_t* pairs, int64_t cap, int64_t* n_pairs) {
    if (!s || !n_pairs || cap < 0 || (cap > 0 && !pairs)) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    if (!s->lists_valid) return s->fail(MD_ERR_STATE, "md_build_neighbors first");
    md_status r = s->hip(md::launch_half_fill(s->sys, s->stream), "half list");
    if (r == MD_OK) r = s->sync_check();
    if (r != MD_OK) return r;
    md::Ctrl c;
    r = s->hip(hipMemcpy(&c, s->sys.ctrl, sizeof c, hipMemcpyDeviceToHost), "ctrl");
    if (r != MD_OK) return r;
    int n = s->p.n;
    std::vector<int> id(n), hs(n + 1), hj((size_t)c.npairs);
    r = s->hip(hipMemcpy(id.data(), s->sys.id, 4 * (size_t)n, hipMemcpyDeviceToHost), "ids");
    if (r == MD_OK)
        r = s->hip(hipMemcpy(hs.data(), s->sys.hstart, 4 * (size_t)(n + 1), hipMemcpyDeviceToHost),
                   "hstart");
    if (r == MD_OK && c.npairs > 0)
        r = s->hip(hipMemcpy(hj.data(), s->sys.hj, 4 * (size_t)c.npairs, hipMemcpyDeviceToHost), "hj");
    if (r != MD_OK) return r;
    *n_pairs = c.npairs;
    int64_t w = 0;
    for (int i = 0; i < n && w < cap; i++)
        for (int k = hs[i]; k < hs[i + 1] && w < cap; k++) {
            int a = id[i], b = id[hj[k] & ((1 << 24) - 1)];  // low 24 bits: slot
            pairs[2 * w] = std::min(a, b);
            pairs[2 * w + 1] = std::max(a, b);
            w++;
        }
    return MD_OK;
}

md_status md_stats(md_system* s, md_stats_t* out) {
    if (!s || !out) return MD_ERR_INVALID_ARG;
    if (s->batch) return s->admitted();
    md_status r = MD_OK;
    if (s->lists_valid) {  // the edge pass's non-zero pairs at the current positions
        r = s->hip(md::launch_half_fill(s->sys, s->stream), "half fill");
        if (r == MD_OK) r = s->hip(md::launch_count_nonzero(s->sys, s->p.prec, s->stream), "count");
        if (r != MD_OK) return r;
    }
    r = s->hip(hipStreamSynchronize(s->stream), "stats sync");
    md::Ctrl c;
    if (r == MD_OK) r = s->hip(hipMemcpy(&c, s->sys.ctrl, sizeof c, hipMemcpyDeviceToHost), "ctrl");
    if (r != MD_OK) return r;
    out->steps = s->steps;
    out->rebuilds = c.rebuilds;
    out->pairs = c.npairs;
    out->max_list_len = c.max_count;
    out->n_cells = s->lay.nc;
    out->tiles_total = s->lay.ntiles;
    out->tiles_staged = c.staged;
    out->nonzero_pairs = s->lists_valid ? c.nonzero : 0;
    return MD_OK;
}

void md_destroy(md_system* s) {
    if (s && s->batch) (void)md_batch_retire(s->batch, s->batch_slot);
    delete s;
}

const char* md_status_str(int32_t status) { return status_text(status); }

const char* md_last_error(const md_system* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched serving (md_batch_*).
// ---------------------------------------------------------------------------

namespace {

struct BatchLayout {
    uint64_t tab = 0, left = 0, map[md::kNumClasses] = {}, bytes = 0;
    int cap[md::kNumClasses] = {};
};

md_status validate_batch(const md_batch_params* p) {
    if (!p) return MD_ERR_INVALID_ARG;
    if (p->max_systems < 1 || p->max_systems > 65536) return MD_ERR_INVALID_ARG;
    if (p->mode != MD_MODE_VERTEX && p->mode != MD_MODE_EDGE && p->mode != MD_MODE_EDGE_DET)
        return MD_ERR_INVALID_ARG;
    if (p->steps_per_launch < 1 || p->steps_per_launch > 4096) return MD_ERR_INVALID_ARG;
    if (p->use_graph != 0 && p->use_graph != 1) return MD_ERR_INVALID_ARG;
    if (p->max_particles < 2 || p->max_particles > (1LL << 30)) return MD_ERR_INVALID_ARG;
    if (p->pool_bytes == 0) return MD_ERR_INVALID_ARG;
    return MD_OK;
}

// Grid capacity of every block class: enough for max_particles spread over
// max_systems systems (each system rounds up once per class).
BatchLayout batch_layout(const md_batch_params& p) {
    BatchLayout L;
    long long nmax = p.max_particles, smax = p.max_systems;
    long long tiles = (nmax + md::kTile - 1) / md::kTile + smax;
    long long c[md::kNumClasses];
    c[md::kClsParticle] = (nmax + md::kBlock - 1) / md::kBlock + smax;
    c[md::kClsTile] = tiles;
    // cell sort: at most nblk blocks per system; tile regions: 4 tiles per block
    c[md::kClsSortTiles] = c[md::kClsParticle] + (tiles + 3) / 4 + smax;
    for (int b = 0; b < md::kLdsBuckets; b++) {
        c[md::kClsVertex0 + b] = tiles;
        c[md::kClsEdge0 + b] = 4 * tiles;
    }
    uint64_t cur = 0;
    L.tab = take(cur, sizeof(md::Sys) * (uint64_t)smax);
    L.left = take(cur, 4 * (uint64_t)smax);
    for (int k = 0; k < md::kNumClasses; k++) {
        L.cap[k] = (int)c[k];
        L.map[k] = take(cur, sizeof(int2) * (uint64_t)c[k]);
    }
    L.bytes = cur;
    return L;
}

// Host twin of the kernels' XCD re-indexing: grid block g runs on XCD g % 8;
// hand each XCD a contiguous range of the class's block list.
int xcd_remap_host(int g, int total) {
    const int nx = 8;
    int q = total / nx, r = total % nx;
    int x = g % nx, k = g / nx;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace

struct md_batch {
    md_batch_params p;
    BatchLayout lay;
    hipStream_t stream = nullptr;   // caller's: uploads and launches
    hipStream_t capture = nullptr;  // private: graph capture only
    md::BatchDev dev{};
    std::vector<md_system*> slot;
    std::vector<long long> left;      // host bookkeeping of steps left
    std::vector<long long> admitted;  // steps requested at admission
    // staging of the device table; written only after the stream is drained
    std::vector<md::Sys> h_tab;
    std::vector<int> h_left;
    std::vector<int2> h_map[md::kNumClasses];
    int used[md::kNumClasses] = {};
    int uploaded[md::kNumClasses] = {};  // map entries that may be non-idle on the device
    int active = 0;
    long long particles = 0;
    uint64_t bytes = 0;
    // Captured launches, one per step count.  Grids are the blocks in use
    // rounded up to a power of two (at least one block, so every kernel of
    // the step is a node); when admissions change them, the kernel nodes of
    // the instantiated graph are re-gridded in place (each node's class from
    // its kernel), so a graph is captured once per step count.
    struct Graph {
        int steps;
        int grid[md::kNumClasses];
        hipGraph_t graph;
        hipGraphExec_t exec;
        std::vector<std::pair<hipGraphNode_t, int>> nodes;  // kernel node, its class
        bool regriddable;  // every node is a known batch kernel
        long long used_at;
    };
    std::vector<Graph> graphs;
    static constexpr size_t kMaxGraphs = 8;
    long long launches = 0, captures = 0, regrids = 0;
    std::string err;

    md_status fail(md_status st, const std::string& msg) {
        err = msg;
        return st;
    }
    md_status hip(hipError_t e, const char* where) {
        if (e == hipSuccess) return MD_OK;
        err = std::string(where) + ": " + hipGetErrorString(e);
        return MD_ERR_HIP;
    }
    void drop_graph(Graph& g) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    void drop_graphs() {
        for (auto& g : graphs) drop_graph(g);
        graphs.clear();
    }
    // Grid of every class for the current admissions: the blocks in use,
    // rounded up to a power of two for captured graphs; a bucket class no
    // admitted system uses gets 0 blocks (not launched) for direct launches
    // and 1 idle block in a graph.
    void grids(bool bucket, int* out) const {
        for (int c = 0; c < md::kNumClasses; c++) {
            bool bucketed = c >= md::kClsVertex0;
            if (bucketed && used[c] == 0) {
                out[c] = bucket ? 1 : 0;
                continue;
            }
            int u = std::max(used[c], 1);
            if (bucket) {
                int g = 1;
                while (g < u) g *= 2;
                u = g;
            }
            out[c] = std::min(u, lay.cap[c]);
        }
    }
    ~md_batch() {
        drop_graphs();
        if (capture) (void)hipStreamDestroy(capture);
    }

    // Rewrites the block maps and uploads table, step budgets and maps.
    // The caller has drained the stream, so the staging buffers are free.
    md_status upload() {
        for (int c = 0; c < md::kNumClasses; c++) {
            std::vector<int2> list;
            list.reserve(used[c]);
            for (int k = 0; k < p.max_systems; k++) {
                if (!slot[k]) continue;
                int nb = md::class_blocks(h_tab[k], c);
                for (int l = 0; l < nb; l++) list.push_back(make_int2(k, l));
            }
            int total = (int)list.size();
            int span = std::max(total, uploaded[c]);
            std::vector<int2>& m = h_map[c];
            m.assign((size_t)span, make_int2(-1, 0));
            for (int g = 0; g < total; g++) m[g] = list[xcd_remap_host(g, total)];
            if (span > 0) {
                md_status r = hip(hipMemcpyAsync((void*)dev.map[c], m.data(), sizeof(int2) * (size_t)span,
                                                 hipMemcpyHostToDevice, stream),
                                  "upload block map");
                if (r != MD_OK) return r;
            }
            uploaded[c] = total;
        }
        for (int k = 0; k < p.max_systems; k++) h_left[k] = slot[k] ? (int)left[k] : 0;
        md_status r = hip(hipMemcpyAsync((void*)dev.tab, h_tab.data(), sizeof(md::Sys) * h_tab.size(),
                                         hipMemcpyHostToDevice, stream),
                          "upload table");
        if (r == MD_OK)
            r = hip(hipMemcpyAsync(dev.left, h_left.data(), 4 * h_left.size(), hipMemcpyHostToDevice,
                                   stream),
                    "upload budgets");
        if (r == MD_OK) r = hip(hipStreamSynchronize(stream), "upload sync");
        return r;
    }

    // Kernel nodes of a captured step with their classes; false if a node is
    // not one of the batch kernels (the graph is then re-captured instead of
    // re-gridded).
    bool collect_nodes(Graph& g) {
        size_t n = 0;
        if (hipGraphGetNodes(g.graph, nullptr, &n) != hipSuccess) return false;
        std::vector<hipGraphNode_t> all(n);
        if (n && hipGraphGetNodes(g.graph, all.data(), &n) != hipSuccess) return false;
        for (hipGraphNode_t node : all) {
            hipGraphNodeType type;
            if (hipGraphNodeGetType(node, &type) != hipSuccess || type != hipGraphNodeTypeKernel)
                return false;
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(node, &kp) != hipSuccess) return false;
            int cls = md::batch_kernel_class(kp.func);
            if (cls == -2) return false;
            if (cls >= 0) g.nodes.emplace_back(node, cls);
        }
        return true;
    }

    // Sets the grid of every node whose class changed; false on failure.
    bool regrid(Graph& g, const int* grid) {
        if (!g.regriddable) return false;
        for (auto& nc : g.nodes) {
            if (g.grid[nc.second] == grid[nc.second]) continue;
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(nc.first, &kp) != hipSuccess) return false;
            kp.gridDim = dim3((unsigned)grid[nc.second]);
            if (hipGraphExecKernelNodeSetParams(g.exec, nc.first, &kp) != hipSuccess) return false;
            if (hipGraphKernelNodeSetParams(nc.first, &kp) != hipSuccess) return false;
        }
        std::copy(grid, grid + md::kNumClasses, g.grid);
        regrids++;
        return true;
    }

    md_status graph_for(int steps, const int* grid, hipGraphExec_t* out) {
        for (size_t k = 0; k < graphs.size(); k++) {
            Graph& g = graphs[k];
            if (g.steps != steps) continue;
            if (!std::equal(grid, grid + md::kNumClasses, g.grid)) {
                // the previous launch of this graph may still run
                md_status r = hip(hipStreamSynchronize(stream), "regrid sync");
                if (r != MD_OK) return r;
                if (!regrid(g, grid)) {  // not re-griddable: capture anew
                    drop_graph(g);
                    graphs.erase(graphs.begin() + k);
                    break;
                }
            }
            g.used_at = launches;
            *out = g.exec;
            return MD_OK;
        }
        if (graphs.size() >= kMaxGraphs) {  // drop the least recently launched
            auto old = std::min_element(graphs.begin(), graphs.end(), [](const Graph& a, const Graph& b) {
                return a.used_at < b.used_at;
            });
            md_status r = hip(hipStreamSynchronize(stream), "graph eviction sync");
            if (r != MD_OK) return r;
            drop_graph(*old);
            graphs.erase(old);
        }
        hipGraph_t graph = nullptr;
        md_status r = hip(hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal), "begin capture");
        if (r != MD_OK) return r;
        hipError_t e = md::launch_batch_steps(dev, grid, p.mode, steps, capture);
        hipError_t e2 = hipStreamEndCapture(capture, &graph);
        r = hip(e != hipSuccess ? e : e2, "capture batch step");
        hipGraphExec_t exec = nullptr;
        if (r == MD_OK) r = hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
        if (r != MD_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        Graph g;
        g.steps = steps;
        std::copy(grid, grid + md::kNumClasses, g.grid);
        g.graph = graph;
        g.exec = exec;
        g.used_at = launches;
        g.regriddable = collect_nodes(g);
        graphs.push_back(std::move(g));
        captures++;
        *out = exec;
        return MD_OK;
    }
};

extern "C" {

md_status md_batch_query_sizes(const md_batch_params* p, uint64_t* workspace_bytes) {
    if (!workspace_bytes) return MD_ERR_INVALID_ARG;
    md_status st = validate_batch(p);
    if (st != MD_OK) return st;
    *workspace_bytes = batch_layout(*p).bytes;
    return MD_OK;
}

md_status md_batch_create(const md_batch_params* p, void* d_workspace, uint64_t workspace_bytes,
                          void* hip_stream, md_batch** out) {
    if (!out) return MD_ERR_INVALID_ARG;
    *out = nullptr;
    md_status st = validate_batch(p);
    if (st != MD_OK) return st;
    if (!d_workspace) return MD_ERR_INVALID_ARG;
    BatchLayout L = batch_layout(*p);
    if (workspace_bytes < L.bytes || (uintptr_t)d_workspace % kAlign) return MD_ERR_BUFFER_TOO_SMALL;
    md_batch* b = new md_batch();
    b->p = *p;
    b->lay = L;
    b->stream = (hipStream_t)hip_stream;
    char* W = (char*)d_workspace;
    b->dev.tab = (const md::Sys*)(W + L.tab);
    b->dev.left = (int*)(W + L.left);
    for (int c = 0; c < md::kNumClasses; c++) b->dev.map[c] = (const int2*)(W + L.map[c]);
    b->dev.nslots = p->max_systems;
    b->slot.assign(p->max_systems, nullptr);
    b->left.assign(p->max_systems, 0);
    b->admitted.assign(p->max_systems, 0);
    b->h_tab.resize(p->max_systems);
    std::memset((void*)b->h_tab.data(), 0, sizeof(md::Sys) * b->h_tab.size());
    b->h_left.assign(p->max_systems, 0);
    st = b->hip(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "capture stream");
    // every map entry idle, every budget zero
    if (st == MD_OK) st = b->hip(hipMemsetAsync(d_workspace, 0, L.bytes, b->stream), "clear batch");
    for (int c = 0; c < md::kNumClasses && st == MD_OK; c++) b->uploaded[c] = L.cap[c];
    if (st == MD_OK) st = b->upload();
    if (st != MD_OK) {
        delete b;
        return st;
    }
    *out = b;
    return MD_OK;
}

md_status md_batch_admit(md_batch* b, md_system* s, int64_t nsteps, int32_t* slot) {
    if (!b || !s || !slot || nsteps < 0 || nsteps > INT32_MAX) return MD_ERR_INVALID_ARG;
    *slot = -1;
    if (s->batch) return b->fail(MD_ERR_STATE, "system already admitted to a batch");
    if (!s->lists_valid) return b->fail(MD_ERR_STATE, "system has no lists (md_build_neighbors)");
    if (b->p.mode == MD_MODE_EDGE_DET && !s->p.edge_store)
        return b->fail(MD_ERR_INVALID_ARG, "the deterministic edge mode needs edge_store = 1");
    int k = 0;
    while (k < b->p.max_systems && b->slot[k]) k++;
    if (k == b->p.max_systems) return b->fail(MD_ERR_BUFFER_TOO_SMALL, "no free slot");
    uint64_t foot = s->lay.state_bytes + s->lay.ws_bytes;
    if (b->bytes + foot > b->p.pool_bytes)
        return b->fail(MD_ERR_BUFFER_TOO_SMALL, "footprint exceeds the pool budget");
    if (b->particles + s->p.n > b->p.max_particles)
        return b->fail(MD_ERR_BUFFER_TOO_SMALL, "particles exceed max_particles");
    for (int c = 0; c < md::kNumClasses; c++)
        if (b->used[c] + md::class_blocks(s->sys, c) > b->lay.cap[c])
            return b->fail(MD_ERR_BUFFER_TOO_SMALL,
                           "block class " + std::to_string(c) + " is full");
    if (!s->forces_valid) {
        md_status r = md_forces(s, b->p.mode);
        if (r != MD_OK) return b->fail(r, std::string("initial forces: ") + s->err);
    }
    md_status r = s->sync_check();
    if (r != MD_OK) return b->fail(r, std::string("system: ") + s->err);
    r = b->hip(hipStreamSynchronize(b->stream), "admit sync");
    if (r != MD_OK) return r;
    b->slot[k] = s;
    b->h_tab[k] = s->sys;
    b->left[k] = nsteps;
    b->admitted[k] = nsteps;
    for (int c = 0; c < md::kNumClasses; c++) b->used[c] += md::class_blocks(s->sys, c);
    b->active++;
    b->particles += s->p.n;
    b->bytes += foot;
    s->batch = b;
    s->batch_slot = k;
    r = b->upload();
    if (r != MD_OK) return r;
    *slot = k;
    return MD_OK;
}

md_status md_batch_step(md_batch* b, int32_t* steps_run) {
    if (!b) return MD_ERR_INVALID_ARG;
    if (steps_run) *steps_run = 0;
    long long need = 0;
    for (int k = 0; k < b->p.max_systems; k++)
        if (b->slot[k]) need = std::max(need, b->left[k]);
    if (need == 0) return MD_OK;
    int steps = b->p.steps_per_launch;
    if (need < steps) {
        steps = 1;
        while (steps < need) steps *= 2;
        steps = std::min(steps, b->p.steps_per_launch);
    }
    md_status r;
    int grid[md::kNumClasses];
    b->grids(b->p.use_graph != 0, grid);
    if (b->p.use_graph) {
        hipGraphExec_t exec = nullptr;
        r = b->graph_for(steps, grid, &exec);
        if (r == MD_OK) r = b->hip(hipGraphLaunch(exec, b->stream), "graph launch");
    } else {
        r = b->hip(md::launch_batch_steps(b->dev, grid, b->p.mode, steps, b->stream),
                   "batch launch");
    }
    if (r != MD_OK) return r;
    for (int k = 0; k < b->p.max_systems; k++)
        if (b->slot[k]) b->left[k] -= std::min<long long>(b->left[k], steps);
    b->launches++;
    if (steps_run) *steps_run = steps;
    return MD_OK;
}

md_status md_batch_steps_left(const md_batch* b, int32_t slot, int64_t* left) {
    if (!b || !left || slot < 0 || slot >= b->p.max_systems) return MD_ERR_INVALID_ARG;
    *left = b->slot[slot] ? b->left[slot] : -1;
    return MD_OK;
}

md_status md_batch_retire(md_batch* b, int32_t slot) {
    if (!b || slot < 0 || slot >= b->p.max_systems) return MD_ERR_INVALID_ARG;
    md_system* s = b->slot[slot];
    if (!s) return b->fail(MD_ERR_INVALID_ARG, "slot is free");
    md_status r = b->hip(hipStreamSynchronize(b->stream), "retire sync");
    if (r != MD_OK) return r;
    for (int c = 0; c < md::kNumClasses; c++) b->used[c] -= md::class_blocks(s->sys, c);
    b->active--;
    b->particles -= s->p.n;
    b->bytes -= s->lay.state_bytes + s->lay.ws_bytes;
    s->steps += b->admitted[slot] - b->left[slot];
    b->slot[slot] = nullptr;
    b->left[slot] = 0;
    b->admitted[slot] = 0;
    std::memset((void*)&b->h_tab[slot], 0, sizeof(md::Sys));
    s->batch = nullptr;
    s->batch_slot = -1;
    r = b->upload();
    if (r != MD_OK) return r;
    return s->sync_check();
}

md_status md_batch_thermostat(md_batch* b, int32_t slot, double temperature, double prob,
                              uint64_t seed, uint64_t counter) {
    if (!b || slot < 0 || slot >= b->p.max_systems) return MD_ERR_INVALID_ARG;
    md_system* s = b->slot[slot];
    if (!s) return b->fail(MD_ERR_INVALID_ARG, "slot is free");
    if (!std::isfinite(temperature) || !(temperature >= 0) || !(prob >= 0) || !(prob <= 1))
        return b->fail(MD_ERR_INVALID_ARG, "thermostat needs temperature >= 0 and 0 <= prob <= 1");
    const double sv = std::sqrt(temperature / s->p.mass);
    const double sl = s->p.pot == MD_POT_PATCHY ? std::sqrt(s->p.inertia * temperature) : 0.0;
    // the system's own arrays (the batch table holds its descriptor), on the
    // batch stream: after the steps launched so far, before the next ones
    return b->hip(md::launch_thermostat(b->h_tab[slot], sv, sl, prob, seed, counter, b->stream),
                  "batch thermostat");
}

md_status md_batch_sync(md_batch* b) {
    if (!b) return MD_ERR_INVALID_ARG;
    return b->hip(hipStreamSynchronize(b->stream), "batch sync");
}

md_status md_batch_info(const md_batch* b, md_batch_info_t* out) {
    if (!b || !out) return MD_ERR_INVALID_ARG;
    out->active = b->active;
    int cap = 0;  // largest LDS bucket in use
    for (int bk = 0; bk < md::kLdsBuckets; bk++)
        if (b->used[md::kClsVertex0 + bk] > 0) cap = md::bucket_cap(bk);
    out->lds_cap = cap;
    out->particles = b->particles;
    out->bytes = b->bytes;
    out->launches = b->launches;
    out->captures = b->captures;
    out->regrids = b->regrids;
    return MD_OK;
}

void md_batch_destroy(md_batch* b) {
    if (!b) return;
    for (int k = 0; k < b->p.max_systems; k++)
        if (b->slot[k]) (void)md_batch_retire(b, k);
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

const char* md_batch_last_error(const md_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
