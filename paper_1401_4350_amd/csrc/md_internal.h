// Internal types shared by the HIP kernels (md_kernels.hip) and the host
// engine (md_engine.hip).  Not part of the public ABI (include/md.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace md {

constexpr int kBlock = 256;  // threads per block of the per-particle kernels
constexpr int kWave = 64;    // CDNA wavefront

// LDS-staged vertex pass: the particles are cut into tiles of kTile
// consecutive slots; for each tile the list build records up to kSegMax slot
// ranges that cover the 27-cell neighbourhoods of its home cells, and list
// entries of the tile index into that concatenation, which the force pass
// copies into LDS with coalesced loads.  Tiles whose region does not fit fall
// back to global gathers.
constexpr int kTile = 64;
constexpr int kTileTpp = kBlock / kTile;  // lanes per particle in the tiled pass
constexpr int kSegMax = 36;
constexpr int kChunkMax = 96;
constexpr int kLdsCapMax = 4096;  // particles per tile region (3 doubles each)
constexpr int kListPadRows = 32;  // spare list rows after the last tile (prefetch reads)
constexpr int kRunPad = 16;       // spare records after the FP32 position copy (list-build reads)

// Device-resident control block (one per system).  Written by kernels, read by
// the host only at syncing calls.
struct Ctrl {
    int rebuild;        // set when a list rebuild is due; cleared by the force pass
    int overflow;       // sticky: a list exceeded its capacity
    int nonfinite;      // sticky: a force or position was NaN/Inf
    int max_count;      // longest full list at the last build
    int staged;         // tiles of the last build whose region fits in LDS
    int pad0;
    long long npairs;   // half-list entries at the last build (clamped to capacity)
    long long rebuilds; // number of builds
    int half_stale;     // the half list predates the last build (filled on demand)
    int eidx_stale;     // the edge index of the full-list entries predates the half list
    long long nonzero;  // half-list entries with a non-zero pair result (md_stats)
    // Fused vertex steps (launch_vertex_kick_drift): a launch with id L whose
    // drift finds a particle past half the skin stores L in req[L & 1]; the
    // next launch, L + 1, does nothing if req[L & 1] == L (its lists would be
    // stale) but store L + 1 in req[(L + 1) & 1], and so on until the host
    // rebuilds and resumes with an id that skips one.
    int req[2];
};

// Completion counters of the kernels whose last workgroup runs an epilogue
// (a scan).  Atomics on one address serialise (about 12 ns each on this
// chip), so workgroup b counts in sub-counter b % kSyncFan (kSyncStride ints
// apart) and the last of each group in a top counter: no counter takes more
// than max(ceil(nb / kSyncFan), kSyncFan) atomics.  All counters are zero
// between launches.
constexpr int kSyncFan = 64;
constexpr int kSyncStride = 16;
constexpr int kSyncInts = (kSyncFan + 1) * kSyncStride;
enum SyncUse { kSyncBin = 0, kSyncBuild, kSyncHalf, kSyncCol, kSyncUses };

// Pair-potential constants in the arithmetic type of the pair maths.
template <typename R>
struct LJc {
    R sig2, eps4, eps24, rc2, vshift;
    R c12, c6;  // 48 eps sigma^12 and 24 eps sigma^6: F/r = r^-2 r^-6 (c12 r^-6 - c6)
};

template <typename R>
struct PatchyC {
    R sig2, eps4, eps24, eps, wca2;  // WCA core
    R eps_p, inv_w2, delta, rpc2;    // patches (rpc2 <= 0: no patch cut-off)
    int model;                       // 0: four patches, WCA, cosine factors; 1: two polar patches
};

// Everything a kernel needs, passed by value.  Particle arrays are packed
// 32-byte records (x, y, z, unused) in cell-sorted slot order.
struct Sys {
    int n;          // particles
    int nc;         // cells per side
    int ncell;      // nc^3
    int cap;        // full-list capacity per particle
    int mcap;       // max(ceil(cap / 4), 2): rows of four 32-bit entries per particle
    int pot;        // 0 LJ, 1 patchy
    int nblk;       // ceil(n / kBlock)
    long long max_half;  // half-list capacity (entries)
    double box, inv_box, cell_inv;  // L, 1/L, nc/L
    double rv2;     // (r_c + r_s)^2
    float rv2_lo, rv2_band;  // FP32 list test: below lo in, from lo + band out, between FP64 decides
    double rc2;     // r_c^2
    double disp2;   // (r_s/2)^2
    double dt, hdt, inv_mass, inv_inertia;
    LJc<double> l64;
    LJc<float> l32;
    PatchyC<double> p64;
    PatchyC<float> p32;

    // state (caller's state buffer)
    double4* pos;
    double4* vel;
    double4* frc;
    double4* quat;   // patchy: (w, x, y, z)
    double4* angm;   // patchy: angular momentum (space frame)
    double4* trq;    // patchy: torque
    int* id;         // slot -> original id

    // workspace
    double4* pos_alt;  // second position buffer (vertex pass with the next drift)
    double4* xbuild;
    double4* tpos;
    float4* tposf;   // FP32 copy of tpos (list-build test)
    double4* tvel;
    double4* tquat;
    double4* tangm;
    int* tid;
    int* cell;
    int* rank;
    int* ccount;
    int* cstart;     // ncell + 1
    int* order;
    int* nbr;        // full lists, tiled (see list_row in the kernels)
    int* ncount;
    int* hcount;
    int* hstart;     // n + 1
    int* hj;         // half-list partner slots, CSR by row
    unsigned* hr;    // tiles with a region: per half-list entry, row in the tile << 16 | region index
    double4* rep;    // Newton mode: nrep replicated force arrays of n records
    int nrep;
    int* chunk_row;  // first row of every 64-pair chunk of the half list
    int* bsum;       // per-block half counts, then offsets
    int* tmax;       // per-tile longest full list of the last build
    // deterministic edge mode (estore != 0): per-edge results and, for every
    // full-list entry, its half-list edge (bit 31 set: the particle is the
    // edge's second member; -1: none), tiled like 32-bit nbr entries
    int estore;
    double4* ef;     // per edge: F on the second member, then (patchy) tau_i, tau_j
    int* eidx;
    int* sync;       // [kSyncUses * kSyncInts] completion counters
    int ntiles;      // ceil(n / kTile)
    int lds_cap;     // region capacity (particles) of a tile staged in LDS
    int4* tile_seg;  // [ntiles * kSegMax]: (slot begin, slot end, LDS base, image code)
    int* tile_nseg;  // segments of the tile, or -1 for global gathers
    int4* tile_chunk;  // [ntiles * kChunkMax]: segments cut into runs of <= kWave slots
    int* tile_nchunk;
    int* tile_row0;  // first home row (z * nc + y) of the tile
    double* epart;   // per-particle potential energy
    double* wpart;   // per-particle virial
    double* fpl;     // LJ edge pass: force planes, component c of slot k at fpl[c * fps + k]
    int fps;         // plane stride (doubles)
    double* kpart;   // per-particle kinetic energy
    double* red;     // reduction partials (3 * kRedBlocks) + result (3)
    Ctrl* ctrl;
    int cell_order;  // md_cell_order; nonzero: no tile staged in LDS
    const int* cell_rank;  // curve orders: cell id of row-major cell (z * nc + y) * nc + x
    int prec;        // md_precision of the pair maths
    int launch_id;   // fused vertex steps: id of this launch (see Ctrl::req)
    int* host_run;   // fused vertex steps: host-mapped word, gets the id of every launch that runs
};

constexpr int kRedBlocks = 1024;

// ---------------------------------------------------------------------------
// Batched step.  A batch runs many independent systems through one fixed
// kernel sequence per step.  Each kernel of the sequence belongs to a block
// class that fixes how many blocks a system gets in it; a per-class map sends
// every block of the grid (at least the blocks in use, at most the class's
// capacity) to (slot, block of that system), or to -1 for an idle block.  A
// block never serves two systems, so a system's arithmetic does not depend on
// the others in the batch.
// ---------------------------------------------------------------------------
enum BatchClass {
    kClsParticle = 0,  // nblk = ceil(n / kBlock)
    kClsTile,          // ntiles (one block per tile of kTile slots)
    kClsSortTiles,     // nblk + ceil(ntiles / 4): cell sort, then a wavefront per tile
    // Kernels that stage or accumulate over a tile's region in LDS come in
    // three LDS buckets, each launched with its own fixed dynamic LDS, so a
    // few small-box systems with large regions do not lower the occupancy of
    // all the others.  A system's blocks go to the bucket of its region
    // capacity (lds_bucket); its count in the other two is zero.
    kClsVertex0,       // vertex pass: LJ ntiles; patchy ntiles or nblk (patchy_vertex_tpp)
    kClsVertex1,
    kClsVertex2,
    kClsEdge0,         // edge pass: one block per tile
    kClsEdge1,
    kClsEdge2,
    kNumClasses
};

constexpr int kLdsBuckets = 3;

// Largest region capacity (slots) of each LDS bucket: with 24-byte records,
// bucket 0 leaves room for four workgroups per CU, bucket 1 for three.
__host__ __device__ constexpr int bucket_cap(int b) {
    return b == 0 ? 1664 : (b == 1 ? 2240 : kLdsCapMax);
}

__host__ __device__ inline int lds_bucket(const Sys& s) {
    if (s.pot != 0) return 0;  // the patchy passes use no region
    return s.lds_cap <= bucket_cap(0) ? 0 : (s.lds_cap <= bucket_cap(1) ? 1 : 2);
}

struct BatchDev {
    const Sys* tab;   // [max_systems] descriptors, indexed by slot
    int* left;        // [max_systems] steps left; 0 for free slots
    const int2* map[kNumClasses];  // [cap of the class]: (slot, block) or (-1, 0)
    int nslots;
};

// Workgroups of the cell sort: one lane per particle.
__host__ __device__ inline int sort_blocks(const Sys& s) { return s.nblk; }

// Blocks a system takes in a class.
// Lanes per particle of the patchy vertex pass: kTileTpp up to 65 536
// particles, where one lane per particle leaves most of the chip idle; one
// lane above, where the chip is full and the extra lanes only repeat work.
constexpr int kPatchyLanesMaxN = 65536;
__host__ __device__ inline int patchy_vertex_tpp(const Sys& s) {
    return s.n <= kPatchyLanesMaxN ? kTileTpp : 1;
}

__host__ __device__ inline int class_blocks(const Sys& s, int cls) {
    switch (cls) {
        case kClsParticle: return s.nblk;
        case kClsTile: return s.ntiles;
        case kClsSortTiles: return sort_blocks(s) + (s.ntiles + kBlock / kWave - 1) / (kBlock / kWave);
        case kClsVertex0: case kClsVertex1: case kClsVertex2:
            return lds_bucket(s) == cls - kClsVertex0
                       ? (s.pot == 0 || patchy_vertex_tpp(s) > 1 ? s.ntiles : s.nblk)
                       : 0;
        default:
            return lds_bucket(s) == cls - kClsEdge0 ? s.ntiles : 0;
    }
}

// Enqueues `steps` batched steps (forces by `mode`) plus the step-count
// update on `st`; the kernels of class c get grid[c] blocks (at most the map
// capacity of the class, at least the blocks in use; a class with no blocks
// is not launched).
hipError_t launch_batch_steps(const BatchDev& b, const int* grid, int mode, int steps,
                              hipStream_t st);
// Block class of a kernel of the batched step (by its host function): the
// class whose grid it is launched with, -1 for a kernel of fixed grid, -2 for
// a function that is not one of them.  Lets a captured step be re-gridded in
// place when admissions change the blocks in use.
int batch_kernel_class(const void* func);

// Host-side launchers (md_kernels.hip).  All enqueue on `st`.
hipError_t launch_set_rebuild(const Sys& s, hipStream_t st);
hipError_t launch_clear_ctrl(const Sys& s, hipStream_t st);
hipError_t launch_rebuild(const Sys& s, hipStream_t st, bool cells, bool lists);
// Fills the half list if the last build made it stale (returns at once
// otherwise); the edge and Newton passes and the pair download need it.
hipError_t launch_half_fill(const Sys& s, hipStream_t st);
// With kick, `mid` (if not null) is recorded between the force kernels and
// a separate closing kick kernel (after the force kernel when the kick is
// fused into it).
hipError_t launch_forces(const Sys& s, int mode, int prec, bool kick, hipStream_t st,
                         int edge_grid, hipEvent_t mid = nullptr);
hipError_t launch_kick_drift(const Sys& s, bool zero_forces, hipStream_t st);
// LJ vertex forces with the closing half kick and the next step's half kick,
// drift (into pos_alt) and rebuild test.
hipError_t launch_vertex_kick_drift(const Sys& s, int prec, hipStream_t st);
hipError_t launch_kick(const Sys& s, hipStream_t st);
hipError_t launch_energy(const Sys& s, int prec, hipStream_t st);
// Counts into ctrl->nonzero (cleared first) the half-list entries whose pair
// result is non-zero at the current positions; needs a filled half list.
hipError_t launch_count_nonzero(const Sys& s, int prec, hipStream_t st);
hipError_t launch_clear_rebuild(const Sys& s, hipStream_t st);

// Momentum refresh of the NVT thermostat (sv = sqrt(T / m), sl = sqrt(I T)).
hipError_t launch_thermostat(const Sys& s, double sv, double sl, double prob, uint64_t seed,
                             uint64_t counter, hipStream_t st);

// md_forces_static: zero n ints (a fill kernel, no memset node); load the
// caller's device coordinates (and quaternions) into the slot records; store
// forces (and torques, if t is not null) back in original order; write the
// sticky error of the call (or 0) to *out.
hipError_t launch_fill_zero(int* p, long long n, hipStream_t st);
hipError_t launch_load_records(const Sys& s, const double* x, const double* q, hipStream_t st);
hipError_t launch_store_results(const Sys& s, double* f, double* t, hipStream_t st);
hipError_t launch_status(const Sys& s, int* out, int overflow_code, int nonfinite_code,
                         hipStream_t st);

// Fills the potential constants of s from the physical parameters.
void set_potential(Sys& s, double eps, double sigma, double rc, double eps_p, double w,
                   double delta, double rpc, int patch_model);

}  // namespace md
