// Tracklet binning for gfx950.
//
// Every tracklet gets an exact cell key (group, chamber, dy bin, y bin, pad
// row); the tracklets are then ordered by (key, input index) with a stable
// least-significant-digit radix sort over 8-bit digits that carries the
// 16-byte search record (y, dy, z, input index) along.  Digit histograms
// live in LDS, ranks come from wavefront ballots, so there are no global
// atomics.  Cell offsets follow from the run boundaries of the sorted keys
// and a suffix minimum.  The search road of a track is then a few contiguous
// record ranges, one per (stack, dy bin, y bin) holding all its pad rows: the
// covariance road of Sect. 3 of the paper, enumerated through the cells it
// overlaps.
#include "trd_internal.h"

namespace trd {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;                  // counts per thread in the scans
constexpr int kScanTile = kBlock * kScanItems;  // counts per workgroup
constexpr int kRadixBits = 8;
constexpr int kBins = 1 << kRadixBits;          // 256 digit values
constexpr int kSub = 8;                         // sub-tiles of 256 elements per block
constexpr int kSortTile = kBlock * kSub;        // elements per radix workgroup

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
    // bins in double: the float value widened, a power-of-two scale, floor
    const double u = floor(((double)y - b.y_min) * b.inv_w);
    const int yb = !(u >= 0.0) ? 0 : (u > (double)(b.n_yb - 1) ? b.n_yb - 1 : (int)u);
    const double v = floor(((double)dy - b.dy_min) * b.inv_wd);
    const int db = !(v >= 0.0) ? 0 : (v > (double)(b.n_db - 1) ? b.n_db - 1 : (int)v);
    return ((((uint32_t)grp * kDet + det) * (uint32_t)b.n_db + (uint32_t)db) * (uint32_t)b.n_yb +
            (uint32_t)yb) * (uint32_t)b.n_rows + row;
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

// Source of the radix passes: the caller's tracklet arrays on the first
// pass (key computed on the fly), the previous pass's output afterwards.
struct RadixSrc {
    const float *y, *z, *dy;
    const uint32_t *det_row;
    const int32_t *grp;
    const uint32_t *keys;  // null on the first pass
    const float4 *recs;
};

__device__ __forceinline__ void radix_load(const RadixSrc &src, const BinCfg &b, int64_t e,
                                           uint32_t &key, float4 &rec)
{
    if (src.keys) {
        key = src.keys[e];
        rec = src.recs[e];
    } else {
        const float y = src.y[e], z = src.z[e], dy = src.dy[e];
        key = cell_key(y, z, dy, src.det_row[e], src.grp ? src.grp[e] : 0, b);
        rec = make_float4(y, dy, z, __int_as_float((int)e));
    }
}

__device__ __forceinline__ uint32_t radix_key_only(const RadixSrc &src, const BinCfg &b, int64_t e)
{
    if (src.keys) return src.keys[e];
    return cell_key(src.y[e], src.z[e], src.dy[e], src.det_row[e], src.grp ? src.grp[e] : 0, b);
}

// digit histogram of one tile, stored digit-major: hist[d * n_blocks + block]
__global__ void __launch_bounds__(kBlock)
    k_radix_hist(RadixSrc src, BinCfg b, int64_t n, int shift, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[kBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kBlock + threadIdx.x;
        if (e < n) atomicAdd(&h[(radix_key_only(src, b, e) >> shift) & (kBins - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: elements are taken in input order (sub-tile,
// wavefront, lane); a lane's rank among equal digits of its wavefront comes
// from eight ballots, the counts of earlier wavefronts and sub-tiles from LDS.
// The tile is first regrouped by digit in LDS, so that each digit's run goes
// out as contiguous stores.
__global__ void __launch_bounds__(kBlock)
    k_radix_scatter(RadixSrc src, BinCfg b, int64_t n, int shift, const uint32_t *__restrict__ hist,
                    const uint32_t *__restrict__ hist_off, uint32_t *__restrict__ keys_out,
                    float4 *__restrict__ recs_out)
{
    __shared__ uint32_t run[kBins];      // elements of each digit placed so far in this tile
    __shared__ uint32_t loc[kBins];      // first LDS slot of each digit in this tile
    __shared__ uint32_t glob[kBins];     // first global position of each digit for this tile
    __shared__ uint32_t wcnt[kBlock / 64][kBins];
    __shared__ uint32_t skey[kSortTile];
    __shared__ float4 srec[kSortTile];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t cnt = hist[(int64_t)tid * gridDim.x + blockIdx.x];
    uint32_t tot;
    loc[tid] = block_excl_scan(cnt, &tot);
    glob[tid] = hist_off[(int64_t)tid * gridDim.x + blockIdx.x];
    run[tid] = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; w++) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kBlock + tid;
        const bool valid = e < n;
        uint32_t key = 0;
        float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) radix_load(src, b, e, key, rec);
        const uint32_t d = (key >> shift) & (kBins - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kRadixBits; bit++) {
            const uint64_t m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t r = run[d] + rank;
            for (int w = 0; w < wv; w++) r += wcnt[w][d];
            skey[loc[d] + r] = key;
            srec[loc[d] + r] = rec;
        }
        __syncthreads();
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; w++) {
            t += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += t;
        __syncthreads();
    }
    // slot p holds the (p - loc[d])-th element of digit d in this tile
    const int nv = (int)tot;
    for (int p = tid; p < nv; p += kBlock) {
        const uint32_t key = skey[p];
        const uint32_t d = (key >> shift) & (kBins - 1);
        const uint32_t pos = glob[d] + (uint32_t)p - loc[d];
        keys_out[pos] = key;
        recs_out[pos] = srec[p];
    }
}

// first sorted position of each key: offsets[key[p]] = p at run starts
__global__ void __launch_bounds__(kBlock)
    k_run_starts(const uint32_t *__restrict__ keys, int64_t n, uint32_t *__restrict__ offsets)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t k = keys[p];
    if (p == 0 || keys[p - 1] != k) offsets[k] = (uint32_t)p;
}

// load the kScanItems values owned by this thread (pad past the end)
__device__ __forceinline__ void load_items(const uint32_t *in, int64_t n, int64_t base, uint32_t pad,
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
        for (int j = 0; j < kScanItems; j++) v[j] = (base + j < n) ? in[base + j] : pad;
    }
}

// store the kScanItems values owned by this thread (nothing past the end)
__device__ __forceinline__ void store_items(uint32_t *out, int64_t n, int64_t base,
                                            const uint32_t (&v)[kScanItems])
{
    if (base + kScanItems <= n) {
        uint4 *q = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; j++)
            q[j] = make_uint4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; j++)
            if (base + j < n) out[base + j] = v[j];
    }
}

__global__ void __launch_bounds__(kBlock)
    k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, uint32_t *__restrict__ block_sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(in, n, base, 0u, v);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) s += v[j];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the per-tile sums in place
__global__ void __launch_bounds__(kBlock) k_scan_top(uint32_t *__restrict__ sums, int64_t nb)
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
}

__global__ void __launch_bounds__(kBlock)
    k_scan_down(const uint32_t *__restrict__ in, int64_t n, const uint32_t *__restrict__ tile_off,
                uint32_t *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(in, n, base, 0u, v);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) s += v[j];
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + tile_off[blockIdx.x];
    uint32_t o[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        o[j] = run;
        run += v[j];
    }
    store_items(out, n, base, o);
}

// ---- suffix minimum (offsets of empty cells = start of the next run) ----

__device__ __forceinline__ uint32_t wave_suffix_min(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_down(v, d, 64);
        if (lane + d < 64) v = t < v ? t : v;
    }
    return v;
}

// inclusive suffix minimum over the workgroup, given each thread's value
__device__ __forceinline__ uint32_t block_suffix_min(uint32_t v)
{
    __shared__ uint32_t wmin[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t s = wave_suffix_min(v);
    if (lane == 0) wmin[wid] = s;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kBlock / 64; w++)
        if (w > wid) s = wmin[w] < s ? wmin[w] : s;
    __syncthreads();
    return s;
}

// value held by thread tid + 1 of the workgroup (all-ones for the last one)
__device__ __forceinline__ uint32_t block_next(uint32_t v)
{
    __shared__ uint32_t firsts[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t nx = __shfl_down(v, 1, 64);
    if (lane == 0) firsts[wid] = v;
    __syncthreads();
    if (lane == 63) nx = wid + 1 < kBlock / 64 ? firsts[wid + 1] : 0xffffffffu;
    __syncthreads();
    return nx;
}

__global__ void __launch_bounds__(kBlock)
    k_min_reduce(const uint32_t *__restrict__ in, int64_t n, uint32_t *__restrict__ tile_min)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(in, n, base, 0xffffffffu, v);
    uint32_t m = 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) m = v[j] < m ? v[j] : m;
    m = block_suffix_min(m);
    if (threadIdx.x == 0) tile_min[blockIdx.x] = m;
}

// one workgroup: each tile minimum becomes the minimum over the later tiles
__global__ void __launch_bounds__(kBlock) k_min_top(uint32_t *__restrict__ mins, int64_t nb)
{
    __shared__ uint32_t head;
    uint32_t carry = 0xffffffffu;
    const int64_t nchunks = (nb + kBlock - 1) / kBlock;
    for (int64_t c = nchunks - 1; c >= 0; c--) {
        const int64_t i = c * kBlock + threadIdx.x;
        const uint32_t v = i < nb ? mins[i] : 0xffffffffu;
        const uint32_t incl = block_suffix_min(v);
        const uint32_t nx = block_next(incl);
        if (i < nb) mins[i] = nx < carry ? nx : carry;
        if (threadIdx.x == 0) head = incl;
        __syncthreads();
        carry = head < carry ? head : carry;
        __syncthreads();
    }
}

// in place: each value becomes the minimum of itself and everything after it
__global__ void __launch_bounds__(kBlock)
    k_min_down(uint32_t *__restrict__ a, int64_t n, const uint32_t *__restrict__ tile_after)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(a, n, base, 0xffffffffu, v);
    uint32_t m = 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) m = v[j] < m ? v[j] : m;
    const uint32_t nx = block_next(block_suffix_min(m));  // later threads of this tile
    const uint32_t t = tile_after[blockIdx.x];            // later tiles
    uint32_t run = nx < t ? nx : t;
#pragma unroll
    for (int j = kScanItems - 1; j >= 0; j--) {
        run = v[j] < run ? v[j] : run;
        v[j] = run;
    }
    store_items(a, n, base, v);
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

int64_t scan_block_sums_len(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }
int64_t radix_blocks(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// exclusive sum scan of n values (out may alias nothing of in)
static void launch_excl_scan(const uint32_t *in, int64_t n, uint32_t *tiles, uint32_t *out,
                             hipStream_t s)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) return;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, tiles, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tiles, out);
}

// in-place inclusive suffix minimum of n values
static void launch_suffix_min(uint32_t *a, int64_t n, uint32_t *tiles, hipStream_t s)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) return;
    hipLaunchKernelGGL(k_min_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, a, n, tiles);
    hipLaunchKernelGGL(k_min_top, dim3(1), dim3(kBlock), 0, s, tiles, nb);
    hipLaunchKernelGGL(k_min_down, dim3((unsigned)nb), dim3(kBlock), 0, s, a, n, tiles);
}

void launch_bin(const float *y, const float *z, const float *dy, const uint32_t *det_row,
                const int32_t *grp, int64_t n, const BinCfg &b, BinBuffers &buf, hipStream_t s)
{
    const int64_t nc = (int64_t)b.n_cells;
    // offsets: n for the end sentinel, "none" elsewhere until run starts fill in
    launch_fill_u32(buf.offsets, 0xffffffffu, nc, s);
    launch_fill_u32(buf.offsets + nc, (uint32_t)n, 1, s);
    if (n > 0) {
        int bits = 1;
        while (bits < 32 && (uint64_t)nc >> bits) bits++;
        const int passes = (bits + kRadixBits - 1) / kRadixBits;
        const int64_t nblk = radix_blocks(n);
        // ping-pong so that the last pass lands in buf.sorted
        uint32_t *kdst[2] = {buf.keys_a, buf.keys_b};
        float4 *rdst[2] = {buf.sorted, buf.recs_tmp};
        int out = (passes % 2 == 1) ? 0 : 1;
        RadixSrc src{y, z, dy, det_row, grp, nullptr, nullptr};
        for (int p = 0; p < passes; p++) {
            const int shift = p * kRadixBits;
            hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(kBlock), 0, s, src, b, n, shift,
                               buf.hist);
            launch_excl_scan(buf.hist, nblk * kBins, buf.tiles_tkl, buf.hist_off, s);
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, s, src, b, n, shift,
                               buf.hist, buf.hist_off, kdst[out], rdst[out]);
            src.keys = kdst[out];
            src.recs = rdst[out];
            out ^= 1;
        }
        hipLaunchKernelGGL(k_run_starts, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, src.keys, n,
                           buf.offsets);
        buf.sorted_keys = src.keys;
    }
    launch_suffix_min(buf.offsets, nc + 1, buf.tiles_cell, s);
}

}  // namespace trd
