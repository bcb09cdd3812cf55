// Tracklet binning for gfx950.
//
// Every tracklet gets an exact cell key (group, chamber, dy bin, y bin, pad
// row); the tracklets are then ordered by (key, input index) with a stable
// least-significant-digit radix sort over 8-bit digits that carries the
// 16-byte search record (y, dy, z, input index) along.  Digit histograms
// live in LDS, ranks come from wavefront ballots, so there are no global
// atomics.  Cell offsets follow from the run boundaries of the sorted keys,
// every cell written once.  The search road of a track is then a few contiguous
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
        !__builtin_isfinite(y) || !__builtin_isfinite(z) || !__builtin_isfinite(dy) || slot_absent(b, (int)det))
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

// Sources of the radix passes.  First pass of the tracklet sort: the
// caller's arrays, key and record computed on the fly.  Later passes (and
// any sort of precomputed keys): the previous pass's keys and records.
struct TklSrc {
    const float *y, *z, *dy;
    const uint32_t *det_row;
    const int32_t *grp;
    BinCfg b;
    const uint32_t *cached;  // keys written by the histogram pass (null there)
    using Rec = float4;
    __device__ __forceinline__ uint32_t key(int64_t e) const
    {
        return cell_key(y[e], z[e], dy[e], det_row[e], grp ? grp[e] : 0, b);
    }
    __device__ __forceinline__ void load(int64_t e, uint32_t &k, float4 &rec) const
    {
        const float ye = y[e], ze = z[e], dye = dy[e];
        k = cached ? cached[e] : cell_key(ye, ze, dye, det_row[e], grp ? grp[e] : 0, b);
        rec = make_float4(ye, dye, ze, __int_as_float((int)e));
    }
};

// First pass of the track sort: the seed's order key, its index as value.
template <typename TS>
struct TrkSrc {
    const TS *ip;
    const int32_t *isec, *igrp;
    int64_t n;
    int32_t n_groups;
    using Rec = uint32_t;
    __device__ __forceinline__ uint32_t key(int64_t e) const
    {
        return track_order_key(ip[e], ip[n + e], ip[4 * n + e], isec[e], igrp ? igrp[e] : 0, n_groups);
    }
    __device__ __forceinline__ void load(int64_t e, uint32_t &k, uint32_t &rec) const
    {
        k = key(e);
        rec = (uint32_t)e;
    }
};

template <typename R>
struct PassSrc {
    const uint32_t *keys;
    const R *recs;
    using Rec = R;
    __device__ __forceinline__ uint32_t key(int64_t e) const { return keys[e]; }
    __device__ __forceinline__ void load(int64_t e, uint32_t &k, R &rec) const
    {
        k = keys[e];
        rec = recs[e];
    }
};

// digit histogram of one tile, stored digit-major: hist[d * n_blocks + block]
template <typename Src>
__global__ void __launch_bounds__(kBlock)
    k_radix_hist(Src src, int64_t n, int shift, uint32_t *__restrict__ hist, uint32_t *__restrict__ key_out)
{
    __shared__ uint32_t h[kBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kBlock + threadIdx.x;
        if (e < n) {
            const uint32_t k = src.key(e);
            if (key_out) key_out[e] = k;
            atomicAdd(&h[(k >> shift) & (kBins - 1)], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: elements are taken in input order (sub-tile,
// wavefront, lane).  Each wavefront ranks its lanes among equal digits with
// eight ballots and records, per sub-tile, the count of each digit it holds;
// one pass over those counts per digit turns them into the offsets of each
// (sub-tile, wavefront) within the digit's run, so the whole tile is ranked
// with four barriers.  The tile is regrouped by digit in LDS, so that each
// digit's run goes out as contiguous stores.
template <typename Src>
__global__ void __launch_bounds__(kBlock)
    k_radix_scatter(Src src, int64_t n, int shift, const uint32_t *__restrict__ hist,
                    const uint32_t *__restrict__ hist_off, uint32_t *__restrict__ keys_out,
                    typename Src::Rec *__restrict__ recs_out, uint32_t *__restrict__ rank_out)
{
    using Rec = typename Src::Rec;
    constexpr int kWaves = kBlock / 64;
    __shared__ uint32_t loc[kBins];                  // first LDS slot of each digit in this tile
    __shared__ uint32_t glob[kBins];                 // first global position of each digit for this tile
    __shared__ uint16_t cnt[kSub * kWaves][kBins];   // per (sub-tile, wavefront): count, then offset
    __shared__ uint32_t skey[kSortTile];
    __shared__ Rec srec[kSortTile];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t hc = hist[(int64_t)tid * gridDim.x + blockIdx.x];
    uint32_t tot;
    loc[tid] = block_excl_scan(hc, &tot);
    glob[tid] = hist_off[(int64_t)tid * gridDim.x + blockIdx.x];
#pragma unroll
    for (int q = 0; q < kSub * kWaves; q++) cnt[q][tid] = 0;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    // all of this thread's elements in flight at once
    uint32_t kv[kSub];
    Rec rv[kSub];
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kBlock + tid;
        kv[j] = 0;
        rv[j] = Rec{};
        if (e < n) src.load(e, kv[j], rv[j]);
    }
    __syncthreads();
    // rank within the wavefront; the first lane of each digit records its count
    uint32_t rk[kSub];
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const bool valid = base + j * kBlock + tid < n;
        const uint32_t d = (kv[j] >> shift) & (kBins - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kRadixBits; bit++) {
            const uint64_t m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        rk[j] = (uint32_t)__popcll(peers & lt);
        if (valid && rk[j] == 0) cnt[j * kWaves + wv][d] = (uint16_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: counts in (sub-tile, wavefront) order -> exclusive offsets
    {
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kSub * kWaves; q++) {
            const uint32_t c = cnt[q][tid];
            cnt[q][tid] = (uint16_t)run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        if (base + j * kBlock + tid < n) {
            const uint32_t d = (kv[j] >> shift) & (kBins - 1);
            const uint32_t slot = loc[d] + cnt[j * kWaves + wv][d] + rk[j];
            skey[slot] = kv[j];
            srec[slot] = rv[j];
        }
    }
    __syncthreads();
    // slot p holds the (p - loc[d])-th element of digit d in this tile
    const int nv = (int)tot;
    for (int p = tid; p < nv; p += kBlock) {
        const uint32_t key = skey[p];
        const uint32_t d = (key >> shift) & (kBins - 1);
        const uint32_t pos = glob[d] + (uint32_t)p - loc[d];
        keys_out[pos] = key;
        recs_out[pos] = srec[p];
        // last pass of an index sort: where each index ended up
        if constexpr (sizeof(Rec) == 4)
            if (rank_out) rank_out[srec[p]] = pos;
    }
}

// Cell offsets from the sorted keys in one pass: offsets[c] is the first
// sorted position whose key is >= c, for c in [0, n_cells].  Position p
// (0 <= p <= n, with p = n standing for the end) owns the cells
// (key[p-1], key[p]] and writes p into each, so every cell is written once.
// Short runs are written by their lane, long runs (empty stretches of the
// detector) by the whole wavefront in turn.
constexpr int64_t kShortRun = 16;
__global__ void __launch_bounds__(kBlock)
    k_offsets(const uint32_t *__restrict__ keys, int64_t n, uint32_t n_cells, uint32_t *__restrict__ offsets)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t lo = 1, hi = 0;
    if (p <= n) {
        lo = p == 0 ? 0 : (int64_t)keys[p - 1] + 1;
        hi = p == n ? (int64_t)n_cells : (int64_t)keys[p];
    }
    const bool is_long = hi - lo + 1 > kShortRun;
    if (!is_long)
        for (int64_t c = lo; c <= hi; c++) offsets[c] = (uint32_t)p;
    uint64_t m = __ballot(is_long);
    const int lane = threadIdx.x & 63;
    while (m) {
        const int src = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int64_t l0 = __shfl(lo, src, 64), h0 = __shfl(hi, src, 64);
        const uint32_t v = (uint32_t)__shfl((int)p, src, 64);
        for (int64_t c = l0 + lane; c <= h0; c += 64) offsets[c] = v;
    }
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

__global__ void __launch_bounds__(kBlock)
    k_scan_down(const uint32_t *__restrict__ in, int64_t n, const uint32_t *__restrict__ tile_sums,
                uint32_t *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(in, n, base, 0u, v);
    // this tile's offset: the sums of the earlier tiles (a few hundred at most)
    uint32_t part = 0;
    for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += kBlock) part += tile_sums[t];
    uint32_t tile_off;
    (void)block_excl_scan(part, &tile_off);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) s += v[j];
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + tile_off;
    uint32_t o[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        o[j] = run;
        run += v[j];
    }
    store_items(out, n, base, o);
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
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tiles, out);
}

// One radix pass from src into (keys_out, recs_out).
template <typename Src>
static void radix_pass(const Src &src, int64_t n, int shift, uint32_t *hist, uint32_t *hist_off,
                       uint32_t *tiles, uint32_t *keys_out, typename Src::Rec *recs_out, hipStream_t s,
                       uint32_t *rank_out = nullptr)
{
    const int64_t nblk = radix_blocks(n);
    hipLaunchKernelGGL(k_radix_hist<Src>, dim3((unsigned)nblk), dim3(kBlock), 0, s, src, n, shift, hist,
                       (uint32_t *)nullptr);
    launch_excl_scan(hist, nblk * kBins, tiles, hist_off, s);
    hipLaunchKernelGGL(k_radix_scatter<Src>, dim3((unsigned)nblk), dim3(kBlock), 0, s, src, n, shift, hist,
                       hist_off, keys_out, recs_out, rank_out);
}

// First pass of the tracklet sort: the histogram pass computes the keys once
// and leaves them in key_cache for the scatter.
static void radix_pass_tkl(TklSrc src, int64_t n, uint32_t *key_cache, uint32_t *hist, uint32_t *hist_off,
                           uint32_t *tiles, uint32_t *keys_out, float4 *recs_out, hipStream_t s)
{
    const int64_t nblk = radix_blocks(n);
    src.cached = nullptr;
    hipLaunchKernelGGL(k_radix_hist<TklSrc>, dim3((unsigned)nblk), dim3(kBlock), 0, s, src, n, 0, hist,
                       key_cache);
    launch_excl_scan(hist, nblk * kBins, tiles, hist_off, s);
    src.cached = key_cache;
    hipLaunchKernelGGL(k_radix_scatter<TklSrc>, dim3((unsigned)nblk), dim3(kBlock), 0, s, src, n, 0, hist,
                       hist_off, keys_out, recs_out, (uint32_t *)nullptr);
}

static int radix_passes(uint64_t max_key)
{
    int bits = 1;
    while (bits < 32 && max_key >> bits) bits++;
    return (bits + kRadixBits - 1) / kRadixBits;
}

void launch_bin(const float *y, const float *z, const float *dy, const uint32_t *det_row,
                const int32_t *grp, int64_t n, const BinCfg &b, BinBuffers &buf, hipStream_t s)
{
    const int64_t nc = (int64_t)b.n_cells;
    const uint32_t *sorted_keys = nullptr;
    if (n > 0) {
        const int passes = radix_passes((uint64_t)nc);
        // ping-pong so that the last pass lands in buf.sorted
        uint32_t *kdst[2] = {buf.keys_a, buf.keys_b};
        float4 *rdst[2] = {buf.sorted, buf.recs_tmp};
        int out = (passes % 2 == 1) ? 0 : 1;
        // the other key buffer is free during the first pass
        radix_pass_tkl(TklSrc{y, z, dy, det_row, grp, b, nullptr}, n, kdst[out ^ 1], buf.hist, buf.hist_off,
                       buf.tiles_tkl, kdst[out], rdst[out], s);
        PassSrc<float4> src{kdst[out], rdst[out]};
        out ^= 1;
        for (int p = 1; p < passes; p++) {
            radix_pass(src, n, p * kRadixBits, buf.hist, buf.hist_off, buf.tiles_tkl, kdst[out], rdst[out], s);
            src = PassSrc<float4>{kdst[out], rdst[out]};
            out ^= 1;
        }
        sorted_keys = src.keys;
    }
    hipLaunchKernelGGL(k_offsets, dim3(grid_for(n + 1, kBlock)), dim3(kBlock), 0, s, sorted_keys, n,
                       (uint32_t)nc, buf.offsets);
}

template <typename TS>
static void track_sort(const TS *ip, const int32_t *isec, const int32_t *igrp, int64_t n, int32_t n_groups,
                       const TrackOrder &o, hipStream_t s)
{
    const int passes = radix_passes((uint64_t)(n_groups * kSectors) << kOrderPosBits);
    uint32_t *kb[2] = {o.key_a, o.key_b};
    uint32_t *vb[2] = {o.val_a, o.val_b};
    radix_pass(TrkSrc<TS>{ip, isec, igrp, n, n_groups}, n, 0, o.hist, o.hist_off, o.tiles, kb[0], vb[0], s,
               passes == 1 ? o.rank : nullptr);
    int cur = 0;
    for (int p = 1; p < passes; p++) {
        radix_pass(PassSrc<uint32_t>{kb[cur], vb[cur]}, n, p * kRadixBits, o.hist, o.hist_off, o.tiles,
                   kb[cur ^ 1], vb[cur ^ 1], s, p == passes - 1 ? o.rank : nullptr);
        cur ^= 1;
    }
}

void launch_track_sort(int precision, const void *ip, const int32_t *isec, const int32_t *igrp, int64_t n,
                       int32_t n_groups, const TrackOrder &o, hipStream_t s)
{
    if (n <= 0) return;
    if (precision == 0)
        track_sort(static_cast<const double *>(ip), isec, igrp, n, n_groups, o, s);
    else
        track_sort(static_cast<const float *>(ip), isec, igrp, n, n_groups, o, s);
}

}  // namespace trd
