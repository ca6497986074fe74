// Device-wide exclusive prefix sums and fill kernels.
//
// Scan: tiles of 2048 int32 (256 threads x 8 consecutive items). Pass 1
// reduces each tile, the tile sums are scanned recursively, and pass 2
// re-reads each tile, scans it in registers (wave shuffles + one LDS step
// across the four waves) and adds the tile's offset. Reads 2x and writes 1x
// the array; used on vertex-sized arrays only, never on the edge stream.
#include "mc_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int64_t SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__global__ __launch_bounds__(SCAN_THREADS) void k_tile_sums(const int32_t* __restrict__ in, int64_t count,
                                                           int32_t* __restrict__ sums) {
    __shared__ int32_t part[SCAN_THREADS / MC_WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        int64_t i = base + k;
        if (i < count) s += in[i];
    }
    s = wave_sum_i32(s);
    if (lane_id() == 0) part[threadIdx.x / MC_WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int k = 0; k < SCAN_THREADS / MC_WAVE; k++) t += part[k];
        sums[blockIdx.x] = t;
    }
}

// Exclusive scan of one tile per block plus the tile offset offs[block]
// (offs == nullptr: 0). The last block also writes out[count].
__global__ __launch_bounds__(SCAN_THREADS) void k_tile_scan(const int32_t* in, int32_t* out, int64_t count,
                                                           const int32_t* __restrict__ offs) {
    __shared__ int32_t wtot[SCAN_THREADS / MC_WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        int64_t i = base + k;
        v[k] = (i < count) ? in[i] : 0;
        tsum += v[k];
    }
    // inclusive scan of thread sums within the wave
    int lane = lane_id();
    int32_t incl = tsum;
    for (int o = 1; o < MC_WAVE; o <<= 1) {
        int32_t y = __shfl_up(incl, o, MC_WAVE);
        if (lane >= o) incl += y;
    }
    if (lane == MC_WAVE - 1) wtot[threadIdx.x / MC_WAVE] = incl;
    __syncthreads();
    int32_t wpre = 0;
    int wid = threadIdx.x / MC_WAVE;
    for (int k = 0; k < wid; k++) wpre += wtot[k];
    int32_t block_total = 0;
    for (int k = 0; k < SCAN_THREADS / MC_WAVE; k++) block_total += wtot[k];
    int32_t off = offs ? offs[blockIdx.x] : 0;
    int32_t run = off + wpre + incl - tsum;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        int64_t i = base + k;
        if (i < count) out[i] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[count] = off + block_total;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_iota_i32(int32_t* p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

inline int grid_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (int)b;
}

}  // namespace

size_t scan_tmp_elems(int64_t count) {
    size_t total = 0;
    int64_t c = count;
    while (c > SCAN_TILE) {
        int64_t nt = (c + SCAN_TILE - 1) / SCAN_TILE;
        total += (size_t)nt + 1;
        c = nt;
    }
    return total + 1;
}

bool scan_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* tmp, hipStream_t s) {
    int64_t nt = (count + SCAN_TILE - 1) / SCAN_TILE;
    if (nt <= 1) {
        k_tile_scan<<<1, SCAN_THREADS, 0, s>>>(in, out, count, nullptr);
        MC_LAUNCHED("k_tile_scan");
        return true;
    }
    int32_t* sums = tmp;
    k_tile_sums<<<(unsigned)nt, SCAN_THREADS, 0, s>>>(in, count, sums);
    MC_LAUNCHED("k_tile_sums");
    if (!scan_i32(sums, sums, nt, tmp + nt + 1, s)) return false;
    k_tile_scan<<<(unsigned)nt, SCAN_THREADS, 0, s>>>(in, out, count, sums);
    MC_LAUNCHED("k_tile_scan");
    return true;
}

bool fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return true;
    k_fill_i32<<<grid_for(count, 256), 256, 0, s>>>(p, v, count);
    MC_LAUNCHED("k_fill_i32");
    return true;
}
bool fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return true;
    k_fill_i64<<<grid_for(count, 256), 256, 0, s>>>(p, v, count);
    MC_LAUNCHED("k_fill_i64");
    return true;
}
bool fill_u8(uint8_t* p, uint8_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return true;
    k_fill_u8<<<grid_for(count, 256), 256, 0, s>>>(p, v, count);
    MC_LAUNCHED("k_fill_u8");
    return true;
}
bool iota_i32(int32_t* p, int64_t count, hipStream_t s) {
    if (count <= 0) return true;
    k_iota_i32<<<grid_for(count, 256), 256, 0, s>>>(p, count);
    MC_LAUNCHED("k_iota_i32");
    return true;
}
