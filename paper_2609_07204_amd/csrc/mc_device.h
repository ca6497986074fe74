// Device-side helpers shared by the HIP kernels of the minimum-cut library:
// the graph record, wave-level reductions, the concurrent union-find used to
// collect contractible edges, and the splitmix64 hash used for start
// vertices. gfx950 only: 64-lane wavefronts throughout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MC_WAVE 64

// Graph on the device in padded-CSR form: row v occupies
// col/w[off[v] .. off[v]+len[v]). Rows are disjoint and may leave gaps, so a
// contraction can write each new row at a position fixed before the merge
// (the total length of the rows it absorbs) without a second compaction.
struct DGraph {
    int32_t n;
    int64_t cap;      // capacity of col/w in entries
    int32_t* off;     // [n]
    int32_t* len;     // [n]
    int32_t* col;     // [cap]
    int64_t* w;       // [cap]
    int64_t* deg;     // [n] weighted degree (sum of the row)
};

// Scalars the host reads back once per round.
struct DevScalars {
    int64_t lam;            // current upper bound on lambda
    int64_t dmin;           // minimum degree of the current graph
    int64_t best_alpha;     // smallest alpha of the last CAPFOREST launch
    unsigned long long marks_pr;
    unsigned long long marks_cf;
    unsigned long long marks_tri;   // of which reduction tests 3 and 4
    int64_t m2;             // entries of the graph the last min_degree read
    int32_t dmin_arg;       // vertex of minimum degree (smallest id on ties)
    int32_t best_pass;      // pass that found best_alpha
    int32_t best_len;       // its scanned-prefix length
    int32_t n2;             // vertex count after relabelling
    int32_t err;            // validation error code (0 = fine)
    int32_t noncanon;       // 1: the input CSR needs the merging normalisation
    int64_t dmax;           // maximum degree of the graph the last min_degree read
    int64_t gmax;           // batched form: the largest total degree of one graph of the batch
};

// ------------------------------------------------------------- atomics
__device__ __forceinline__ int32_t ld_acq(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld64_dev(const int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64_dev(int64_t* p, int64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t atomic_add_i64(int64_t* p, int64_t v) {
    return (int64_t)atomicAdd((unsigned long long*)p, (unsigned long long)v);
}

// ------------------------------------------------------- union-find
// Concurrent union-find over parent[] with the invariant parent[v] <= v:
// a union always hangs the larger root under the smaller one with a CAS, so
// every root is the smallest vertex of its component and finished labels
// are canonical. Finds compress by path halving with plain (relaxed) stores,
// which only ever replace a non-root's parent by one of its ancestors.
// (Jaiganesh and Burtscher, "A high-performance connected components
// implementation for GPUs", HPDC 2018, use the same hooking rule.)
__device__ __forceinline__ int32_t uf_find(int32_t* par, int32_t x) {
    int32_t p = ld_acq(&par[x]);
    if (p == x) return x;
    int32_t prev = x;
    for (;;) {
        int32_t gp = ld_acq(&par[p]);
        if (gp == p) return p;
        st_rel(&par[prev], gp);
        prev = p;
        p = gp;
    }
}

// Returns true if this call joined two different components.
__device__ __forceinline__ bool uf_union(int32_t* par, int32_t a, int32_t b) {
    int32_t ra = uf_find(par, a), rb = uf_find(par, b);
    while (ra != rb) {
        if (ra > rb) { int32_t t = ra; ra = rb; rb = t; }
        int32_t old = atomicCAS(&par[rb], rb, ra);
        if (old == rb) return true;
        rb = uf_find(par, old);
        ra = uf_find(par, ra);
    }
    return false;
}

// ------------------------------------------------------------ hashing
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16; x *= 0x7FEB352Du;
    x ^= x >> 15; x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

// ------------------------------------------------- wave reductions
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int64_t wave_max_i64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}
__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// lexicographic (key descending, id ascending) maximum over the wave;
// entries with id < 0 are empty
__device__ __forceinline__ void wave_argmax(int64_t& key, int32_t& id, int32_t& aux) {
    for (int o = 32; o > 0; o >>= 1) {
        int64_t k2 = __shfl_xor(key, o, 64);
        int32_t i2 = __shfl_xor(id, o, 64);
        int32_t a2 = __shfl_xor(aux, o, 64);
        bool take = (i2 >= 0) && (id < 0 || k2 > key || (k2 == key && i2 < id));
        if (take) { key = k2; id = i2; aux = a2; }
    }
}
// lexicographic (value ascending, id ascending) minimum over the wave
__device__ __forceinline__ void wave_argmin(int64_t& val, int32_t& id) {
    for (int o = 32; o > 0; o >>= 1) {
        int64_t v2 = __shfl_xor(val, o, 64);
        int32_t i2 = __shfl_xor(id, o, 64);
        bool take = (i2 >= 0) && (id < 0 || v2 < val || (v2 == val && i2 < id));
        if (take) { val = v2; id = i2; }
    }
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (MC_WAVE - 1); }

// order and visibility of LDS accesses between the lanes of one wavefront
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------- profiling counters
// Algorithmic-byte counters of the profiled kernels: PROF_LANES counters per
// kernel, 128 B apart, so the once-per-wave adds of a large launch spread
// over many L2 channels instead of queueing on one address. Every lane of
// the wave calls prof_add.
constexpr int PROF_LANES = 64;
constexpr int PROF_STRIDE = 16;   // 16 x 8 B = 128 B
__device__ __forceinline__ void prof_add(unsigned long long* pb, int64_t bytes) {
    bytes = wave_sum_i64(bytes);
    if (lane_id() == 0 && bytes) {
        const unsigned slot = (blockIdx.x * (blockDim.x / MC_WAVE) + threadIdx.x / MC_WAVE) % PROF_LANES;
        atomicAdd(pb + (size_t)slot * PROF_STRIDE, (unsigned long long)bytes);
    }
}
