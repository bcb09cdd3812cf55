// Tracklet binning for gfx950: exact cell keys + histogram, exclusive scan,
// scatter, and a per-cell fix-up that makes the order within a cell the
// input order (so the whole sort is stable and bit-reproducible although
// the scatter slots come from atomics).
//
// Cells are (group, chamber, pad row, y bin); the search road of a track is
// a few contiguous runs of cells (one run of y bins per pad row), which is
// how the covariance road of Sect. 3 of the paper is enumerated.
#include "trd_internal.h"

namespace trd {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;                 // counts per thread
constexpr int kScanTile = kBlock * kScanItems; // counts per workgroup
constexpr int kSmallCell = 32;                 // insertion-sort limit per thread

__global__ void __launch_bounds__(kBlock) k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Cell key of one tracklet; n_cells for the ones that are dropped.
__device__ __forceinline__ uint32_t cell_key(float y, float z, float dy, uint32_t det_row,
                                             int32_t grp, const BinCfg &b)
{
    const uint32_t det = det_row >> 5, row = det_row & 31u;
    if (det >= (uint32_t)kDet || row >= (uint32_t)b.n_rows || grp < 0 || grp >= b.n_groups ||
        !__builtin_isfinite(y) || !__builtin_isfinite(z) || !__builtin_isfinite(dy))
        return b.n_cells;
    // exact in double: y is a float, y_min and 1/w are powers of two times integers
    double u = floor(((double)y - b.y_min) * b.inv_w);
    int yb = u < 0.0 ? 0 : (u > (double)(b.n_yb - 1) ? b.n_yb - 1 : (int)u);
    return (((uint32_t)grp * kDet + det) * (uint32_t)b.n_rows + row) * (uint32_t)b.n_yb +
           (uint32_t)yb;
}

__global__ void __launch_bounds__(kBlock)
    k_key_hist(const float *__restrict__ y, const float *__restrict__ z,
               const float *__restrict__ dy, const uint32_t *__restrict__ det_row,
               const int32_t *__restrict__ grp, int64_t n, BinCfg b, uint32_t *__restrict__ key,
               uint32_t *__restrict__ rank, uint32_t *__restrict__ count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = cell_key(y[i], z[i], dy[i], det_row[i], grp ? grp[i] : 0, b);
    key[i] = k;
    rank[i] = atomicAdd(&count[k], 1u);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan of v over the workgroup; *total receives the sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; w++) {
        off += (w < wid) ? wsum[w] : 0u;
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// load the kScanItems counts owned by this thread (zero past the end)
__device__ __forceinline__ void load_items(const uint32_t *in, int64_t n, int64_t base,
                                           uint32_t (&v)[kScanItems])
{
    if (base + kScanItems <= n) {
        const uint4 *q = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; j++) {
            const uint4 u = q[j];
            v[4 * j] = u.x;
            v[4 * j + 1] = u.y;
            v[4 * j + 2] = u.z;
            v[4 * j + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; j++) v[j] = (base + j < n) ? in[base + j] : 0u;
    }
}

__global__ void __launch_bounds__(kBlock)
    k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, uint32_t *__restrict__ block_sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(in, n, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) s += v[j];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the per-tile sums in place; the grand
// total goes to *total
__global__ void __launch_bounds__(kBlock)
    k_scan_top(uint32_t *__restrict__ sums, int64_t nb, uint32_t *__restrict__ total)
{
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kBlock)
    k_scan_down(const uint32_t *__restrict__ in, int64_t n, const uint32_t *__restrict__ tile_off,
                uint32_t *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(in, n, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) s += v[j];
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + tile_off[blockIdx.x];
    if (base + kScanItems <= n) {
        uint4 *q = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; j++) {
            uint4 u;
            u.x = run; run += v[4 * j];
            u.y = run; run += v[4 * j + 1];
            u.z = run; run += v[4 * j + 2];
            u.w = run; run += v[4 * j + 3];
            q[j] = u;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; j++)
            if (base + j < n) {
                out[base + j] = run;
                run += v[j];
            }
    }
}

__global__ void __launch_bounds__(kBlock)
    k_scatter(const float *__restrict__ y, const float *__restrict__ z,
              const float *__restrict__ dy, const uint32_t *__restrict__ key,
              const uint32_t *__restrict__ rank, const uint32_t *__restrict__ offsets, int64_t n,
              uint32_t n_cells, float4 *__restrict__ sorted)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = key[i];
    if (k >= n_cells) return;  // dropped tracklet
    const uint32_t pos = offsets[k] + rank[i];
    sorted[pos] = make_float4(y[i], dy[i], z[i], __int_as_float((int)i));
}

__device__ __forceinline__ int rec_idx(const float4 &r) { return __float_as_int(r.w); }

// one thread per cell: order the cell's records by input index
__global__ void __launch_bounds__(kBlock)
    k_cell_sort(const uint32_t *__restrict__ offsets, uint32_t n_cells, float4 *__restrict__ sorted,
                uint32_t *__restrict__ big_list, uint32_t *__restrict__ n_big)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const uint32_t a = offsets[c], b = offsets[c + 1];
    if (b - a < 2) return;
    if (b - a > (uint32_t)kSmallCell) {
        big_list[atomicAdd(n_big, 1u)] = (uint32_t)c;
        return;
    }
    for (uint32_t i = a + 1; i < b; i++) {
        const float4 r = sorted[i];
        const int key = rec_idx(r);
        uint32_t j = i;
        while (j > a) {
            const float4 q = sorted[j - 1];
            if (rec_idx(q) <= key) break;
            sorted[j] = q;
            j--;
        }
        sorted[j] = r;
    }
}

// one workgroup per large cell: rank of each record = number of smaller
// input indices in the cell, written through a scratch copy
__global__ void __launch_bounds__(kBlock)
    k_cell_sort_big(const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ big_list,
                    const uint32_t *__restrict__ n_big, float4 *__restrict__ sorted,
                    float4 *__restrict__ tmp)
{
    const uint32_t nb = *n_big;
    for (uint32_t li = blockIdx.x; li < nb; li += gridDim.x) {
        const uint32_t c = big_list[li];
        const uint32_t a = offsets[c], b = offsets[c + 1];
        for (uint32_t e = a + threadIdx.x; e < b; e += blockDim.x) {
            const float4 r = sorted[e];
            const int key = rec_idx(r);
            uint32_t rnk = 0;
            for (uint32_t f = a; f < b; f++) rnk += (rec_idx(sorted[f]) < key) ? 1u : 0u;
            tmp[a + rnk] = r;
        }
        __syncthreads();
        for (uint32_t e = a + threadIdx.x; e < b; e += blockDim.x) sorted[e] = tmp[e];
        __syncthreads();
    }
}

inline unsigned grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kBlock), 0, s, p, v, n);
}

void launch_key_hist(const float *y, const float *z, const float *dy, const uint32_t *det_row,
                     const int32_t *grp, int64_t n, const BinCfg &b, uint32_t *key,
                     uint32_t *rank, uint32_t *count, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_key_hist, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, y, z, dy, det_row,
                       grp, n, b, key, rank, count);
}

int64_t scan_block_sums_len(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_scan(const uint32_t *count, int64_t n, uint32_t *block_sums, uint32_t *offsets,
                 hipStream_t s)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        launch_fill_u32(offsets, 0u, 1, s);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, count, n, block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, block_sums, nb, offsets + n);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, count, n, block_sums,
                       offsets);
}

void launch_scatter(const float *y, const float *z, const float *dy, const uint32_t *key,
                    const uint32_t *rank, const uint32_t *offsets, int64_t n, uint32_t n_cells,
                    float4 *sorted, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, y, z, dy, key, rank,
                       offsets, n, n_cells, sorted);
}

void launch_cell_sort(const uint32_t *offsets, uint32_t n_cells, float4 *sorted, float4 *tmp,
                      uint32_t *big_list, uint32_t *n_big, hipStream_t s)
{
    launch_fill_u32(n_big, 0u, 1, s);
    hipLaunchKernelGGL(k_cell_sort, dim3(grid_for(n_cells, kBlock)), dim3(kBlock), 0, s, offsets,
                       n_cells, sorted, big_list, n_big);
    hipLaunchKernelGGL(k_cell_sort_big, dim3(256), dim3(kBlock), 0, s, offsets, big_list, n_big,
                       sorted, tmp);
}

}  // namespace trd
