// Measurement kernels for the benchmark's rooflines (libmdprobe.so): the
// rates the force passes are held against where the 8 TB/s HBM peak is not
// the whole story -- the edge decomposition is bounded by atomic throughput
// (Methods section: every non-zero pair adds its force with atomics), and the
// achievable HBM read and copy bandwidth.  Not part of the force path; only
// bench.py loads this library.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kBlock = 256;

// A fixed, well-spread slot sequence per thread (splitmix-style mixing of the
// thread and operation index), reduced modulo the slot count.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// kind 0: device-scope FP64 atomic adds at scattered addresses;
// kind 1: the same with the lanes of a wavefront on consecutive addresses.
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_global_atomics(double* buf, int64_t slots, int ops) {
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * kBlock;
    for (int k = 0; k < ops; k++) {
        uint64_t s;
        if (KIND == 0) s = mix64(t * 1315423911ull + (uint64_t)k) % (uint64_t)slots;
        else s = (t + (uint64_t)k * nthreads) % (uint64_t)slots;
        unsafeAtomicAdd(buf + s, 1.0);
    }
}

// LDS FP64 adds inside a workgroup's accumulator of `lslots` doubles, then
// one global store per slot.  KIND 0: atomic adds at scattered addresses;
// 1: atomic adds, the lanes of a wavefront on distinct addresses (stride 37);
// 2: the same addresses with a plain read, add and write (no atomicity: the
// cost of an accumulation whose lanes never collide).
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_lds_atomics(double* out, int lslots, int ops) {
    extern __shared__ double acc[];
    for (int k = threadIdx.x; k < lslots; k += kBlock) acc[k] = 0.0;
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < ops; k++) {
        if (KIND == 0) {
            const int s = (int)(mix64(t * 2654435761ull + (uint64_t)k) % (uint64_t)lslots);
            unsafeAtomicAdd(acc + s, 1.0);
        } else {
            const uint64_t base = mix64((t >> 6) * 2654435761ull + (uint64_t)k);
            const int s = (int)((base + 37u * (uint64_t)lane) % (uint64_t)lslots);
            if (KIND == 1) unsafeAtomicAdd(acc + s, 1.0);
            else acc[s] += 1.0;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < lslots; k += kBlock) out[(size_t)blockIdx.x * lslots + k] = acc[k];
}

// Streaming read of n16 16-byte words, grid-stride, four loads in flight per
// lane; one store per thread keeps the loads live.
typedef int iv4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_read(const iv4* in, int64_t n16, int* out) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    iv4 a = {0, 0, 0, 0};
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const iv4 v0 = __builtin_nontemporal_load(in + i);
        const iv4 v1 = __builtin_nontemporal_load(in + i + stride);
        const iv4 v2 = __builtin_nontemporal_load(in + i + 2 * stride);
        const iv4 v3 = __builtin_nontemporal_load(in + i + 3 * stride);
        a ^= v0 ^ v1 ^ v2 ^ v3;
    }
    for (; i < n16; i += stride) a ^= in[i];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = a.x ^ a.y ^ a.z ^ a.w;
}

}  // namespace

extern "C" {

// Device-scope FP64 atomic adds: `threads` threads (a multiple of 256) each
// add 1.0 `ops` times into buf[0 .. slots), scattered (kind 0) or coalesced
// (kind 1).  buf must hold `slots` doubles.  Async on `stream`.
// Returns 0, or -1 for bad arguments, or the HIP error.
int probe_global_atomics(double* buf, int64_t slots, int64_t threads, int ops, int kind,
                         void* stream) {
    if (!buf || slots < 1 || threads < kBlock || threads % kBlock || ops < 1 ||
        (kind != 0 && kind != 1))
        return -1;
    const dim3 g((unsigned)(threads / kBlock)), b(kBlock);
    hipStream_t st = (hipStream_t)stream;
    if (kind == 0) hipLaunchKernelGGL(k_global_atomics<0>, g, b, 0, st, buf, slots, ops);
    else hipLaunchKernelGGL(k_global_atomics<1>, g, b, 0, st, buf, slots, ops);
    return (int)hipGetLastError();
}

// LDS FP64 adds: `blocks` workgroups of 256 threads, each thread adding 1.0
// `ops` times into its workgroup's LDS accumulator of lslots doubles (64 ..
// 8192): kind 0 atomic at scattered slots, 1 atomic at distinct slots per
// wavefront, 2 plain read-add-write at the same distinct slots.  out
// receives blocks * lslots doubles.
int probe_lds_atomics(double* out, int lslots, int64_t blocks, int ops, int kind, void* stream) {
    if (!out || lslots < 64 * 37 || lslots > 8192 || blocks < 1 || ops < 1 || kind < 0 || kind > 2)
        return -1;
    const dim3 g((unsigned)blocks), b(kBlock);
    const size_t sh = sizeof(double) * (size_t)lslots;
    hipStream_t st = (hipStream_t)stream;
    if (kind == 0) hipLaunchKernelGGL(k_lds_atomics<0>, g, b, sh, st, out, lslots, ops);
    else if (kind == 1) hipLaunchKernelGGL(k_lds_atomics<1>, g, b, sh, st, out, lslots, ops);
    else hipLaunchKernelGGL(k_lds_atomics<2>, g, b, sh, st, out, lslots, ops);
    return (int)hipGetLastError();
}

// Streaming read of `bytes` (a multiple of 16) from in; out receives
// blocks * 256 ints.
int probe_read(const void* in, int64_t bytes, int* out, int64_t blocks, void* stream) {
    if (!in || !out || bytes < 16 || bytes % 16 || blocks < 1) return -1;
    hipLaunchKernelGGL(k_read, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream,
                       (const iv4*)in, bytes / 16, out);
    return (int)hipGetLastError();
}

}  // extern "C"
