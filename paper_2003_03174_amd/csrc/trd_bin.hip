// Tracklet binning for gfx950.
//
// Every tracklet gets an exact cell key (group, chamber, dy bin, y bin, pad
// row); the cells of g consecutive chamber slots form a bucket (key = bucket
// * D + cell of the bucket, D = g * n_db * n_yb * n_rows).  The tracklets are
// then ordered by (key, input index) in two phases that carry the 16-byte
// search record (y, dy, z, input index) along:
//  1. a stable partition by bucket: one pass over an 11-bit digit (up to
//     2047 buckets), then stable 8-bit passes over the higher digits;
//  2. one workgroup per bucket: a stable counting sort of the bucket's
//     tracklets over its D cells in LDS, which also writes the bucket's cell
//     offsets.
// Digit histograms live in LDS and ranks come from wavefront ballots, so
// there are no global atomics.  The search road of a track is then a few
// contiguous record ranges, one per (stack, dy bin, y bin) holding all its
// pad rows: the covariance road of Sect. 3 of the paper, enumerated through
// the cells it overlaps.
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
constexpr int kWideBits = 11;                   // widest digit of the tracklet partition
// threads of its workgroups (tiles of kSub * that many elements): 256 for a
// 10-bit digit, 512 for an 11-bit one (twice the elements per digit and tile;
// 64-frame step 1.45 -> 1.37 ms, while the 10-bit pass of one group loses 5 µs)
template <int kBits> constexpr int kWideThreads = kBits <= 10 ? 256 : 512;

__global__ void __launch_bounds__(kBlock) k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Tile of this workgroup: workgroups are dispatched to the eight XCDs in
// turn (b mod 8), so XCD x takes the x-th contiguous eighth of the tiles and
// the neighbouring tiles' histogram entries meet in one L2.
__device__ __forceinline__ unsigned xcd_tile()
{
    const unsigned nb = gridDim.x, b = blockIdx.x, q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Wavefront-wide ordering of LDS accesses (a wavefront's LDS operations
// complete in issue order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cell key of one tracklet; n_cells for the ones that are dropped.
__device__ __forceinline__ uint32_t cell_key(float y, float z, float dy, uint32_t det_row,
                                             int32_t grp, const BinCfg &b)
{
    // without branches (the absent-slot mask is read at an index kept in
    // bounds), so that the loads of several tracklets can be in flight at once
    const uint32_t det = det_row >> 5, row = det_row & 31u;
    const bool drop = (det >= (uint32_t)kDet) | (row >= (uint32_t)b.n_rows) | (grp < 0) | (grp >= b.n_groups) |
                      !__builtin_isfinite(y) | !__builtin_isfinite(z) | !__builtin_isfinite(dy) |
                      slot_absent(b, det < (uint32_t)kDet ? (int)det : 0);
    // bins in double: the float value widened, a power-of-two scale, floor,
    // clamped to the first and last bin (fmax takes 0 for a NaN)
    const double u = fmin(fmax(floor(((double)y - b.y_min) * b.inv_w), 0.0), (double)(b.n_yb - 1));
    const double v = fmin(fmax(floor(((double)dy - b.dy_min) * b.inv_wd), 0.0), (double)(b.n_db - 1));
    const uint32_t yb = (uint32_t)(int)u, db = (uint32_t)(int)v;
    const uint32_t k = ((((uint32_t)grp * kDet + det) * (uint32_t)b.n_db + db) * (uint32_t)b.n_yb + yb) *
                           (uint32_t)b.n_rows + row;
    const uint32_t m = 0u - (uint32_t)drop;
    return (k & ~m) | (b.n_cells & m);
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

// Bucket of a cell key: key / D, exact (a double estimate, then one integer
// correction).
struct KeyDiv {
    uint32_t c;
    double inv;
    __device__ __forceinline__ uint32_t operator()(uint32_t k) const
    {
        uint32_t q = (uint32_t)((double)k * inv);
        const int64_t r = (int64_t)k - (int64_t)q * c;
        return r < 0 ? q - 1u : (r >= (int64_t)c ? q + 1u : q);
    }
};

// Sources of the sort passes.  Each stores a full key and sorts by
// sort_key(key).  First pass of the tracklet partition: the histogram
// computes each key from the caller's arrays and keeps it, the scatter reads
// that key and builds the record from the caller's arrays, sorted by bucket.
// Later passes: the previous pass's keys and records.
// kGrouped: a group per tracklet in grp (else every tracklet is in group 0
// and grp is not read); a compile-time choice, so that no load is behind a branch
template <bool kGrouped>
struct TklSrc {
    const float *y, *z, *dy;
    const uint32_t *det_row;
    const int32_t *grp;
    BinCfg b;
    KeyDiv slot;
    const uint32_t *cached;  // keys written by the histogram pass, read by the scatter
    using Rec = float4;
    __device__ __forceinline__ uint32_t sort_key(uint32_t k) const { return slot(k); }
    __device__ __forceinline__ uint32_t key(int64_t e) const
    {
        return cell_key(y[e], z[e], dy[e], det_row[e], kGrouped ? grp[e] : 0, b);
    }
    __device__ __forceinline__ void load(int64_t e, uint32_t &k, float4 &rec) const
    {
        k = cached[e];
        rec = make_float4(y[e], dy[e], z[e], __int_as_float((int)e));
    }
};

// First pass of the track sort: the seed's order key, its index as value
// (kGrouped: a group per seed in igrp, else all in group 0 and igrp unread).
template <typename TS, bool kGrouped>
struct TrkSrc {
    const TS *ip;
    const int32_t *isec, *igrp;
    int64_t n;
    int32_t n_groups;
    using Rec = uint32_t;
    __device__ __forceinline__ uint32_t sort_key(uint32_t k) const { return k; }
    __device__ __forceinline__ uint32_t key(int64_t e) const
    {
        return track_order_key(ip[e], ip[n + e], ip[4 * n + e], isec[e], kGrouped ? igrp[e] : 0, n_groups);
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
    __device__ __forceinline__ uint32_t sort_key(uint32_t k) const { return k; }
    __device__ __forceinline__ uint32_t key(int64_t e) const { return keys[e]; }
    __device__ __forceinline__ void load(int64_t e, uint32_t &k, R &rec) const
    {
        k = keys[e];
        rec = recs[e];
    }
};

// later passes of the tracklet partition: still by bucket
struct SlotPassSrc {
    const uint32_t *keys;
    const float4 *recs;
    KeyDiv slot;
    using Rec = float4;
    __device__ __forceinline__ uint32_t sort_key(uint32_t k) const { return slot(k); }
    __device__ __forceinline__ uint32_t key(int64_t e) const { return keys[e]; }
    __device__ __forceinline__ void load(int64_t e, uint32_t &k, float4 &rec) const
    {
        k = keys[e];
        // component-wise: a whole-struct copy puts the caller's record array
        // in scratch memory
        const float4 r = recs[e];
        rec.x = r.x;
        rec.y = r.y;
        rec.z = r.z;
        rec.w = r.w;
    }
};

// digit histogram of one tile, stored digit-major: hist[d * n_blocks + block]
// (only the first nd digits are stored: the ones that occur); tiles of
// kSub * kThreads elements
template <typename Src, int kBits, int kThreads = kBlock>
__global__ void __launch_bounds__(kThreads)
    k_radix_hist(Src src, int64_t n, int shift, int nd, uint32_t *__restrict__ hist, uint32_t *__restrict__ key_out)
{
    constexpr int kNb = 1 << kBits;
    __shared__ uint32_t h[kNb];
    for (int d = threadIdx.x; d < kNb; d += kThreads) h[d] = 0;
    __syncthreads();
    const unsigned tile = xcd_tile();
    const int64_t base = (int64_t)tile * (kSub * kThreads);
    // keys from clamped indexes (n > 0), so that the loads of every
    // sub-tile are in flight together; only the counting is guarded
    uint32_t kv[kSub];
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kThreads + threadIdx.x;
        kv[j] = src.key(e < n ? e : n - 1);
    }
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kThreads + threadIdx.x;
        if (e < n) {
            if (key_out) key_out[e] = kv[j];
            atomicAdd(&h[(src.sort_key(kv[j]) >> shift) & (kNb - 1)], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += kThreads) hist[(int64_t)d * gridDim.x + tile] = h[d];
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
    const unsigned tile = xcd_tile();
    const uint32_t hc = hist[(int64_t)tid * gridDim.x + tile];
    uint32_t tot;
    loc[tid] = block_excl_scan(hc, &tot);
    glob[tid] = hist_off[(int64_t)tid * gridDim.x + tile];
#pragma unroll
    for (int q = 0; q < kSub * kWaves; q++) cnt[q][tid] = 0;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)tile * kSortTile;
    // all of this thread's elements in flight at once (clamped indexes,
    // n > 0; the lanes past the end take no part below)
    uint32_t kv[kSub];
    Rec rv[kSub];
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kBlock + tid;
        src.load(e < n ? e : n - 1, kv[j], rv[j]);
    }
    __syncthreads();
    // rank within the wavefront; the first lane of each digit records its count
    uint32_t rk[kSub];
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const bool valid = base + j * kBlock + tid < n;
        const uint32_t d = (src.sort_key(kv[j]) >> shift) & (kBins - 1);
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
            const uint32_t d = (src.sort_key(kv[j]) >> shift) & (kBins - 1);
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
        const uint32_t d = (src.sort_key(key) >> shift) & (kBins - 1);
        const uint32_t pos = glob[d] + (uint32_t)p - loc[d];
        keys_out[pos] = key;
        recs_out[pos] = srec[p];
        // last pass of an index sort: where each index ended up
        if constexpr (sizeof(Rec) == 4)
            if (rank_out) rank_out[srec[p]] = pos;
    }
}

// Stable scatter of one tile over a wide digit (kBits of 10 or 11): too
// many digits for per-(sub-tile, wavefront) count tables, so the sub-tiles
// go one after the other.  In each, a wavefront ranks its lanes among equal
// digits with ballots and the first lane of each digit posts the count; a
// lane's position is then the digit's start for this tile + what earlier
// sub-tiles placed + what earlier wavefronts of this sub-tile hold + its
// rank.  Two barriers per sub-tile.  With a few elements per digit and tile
// there is nothing to gain from regrouping the tile in LDS before the
// stores, so each lane stores its element directly (and the small LDS
// footprint keeps many workgroups resident).
template <typename Src, int kBits, int kThreads>
__global__ void __launch_bounds__(kThreads)
    k_wide_scatter(Src src, int64_t n, int shift, int nd, const uint32_t *__restrict__ hist_off,
                   uint32_t *__restrict__ keys_out, typename Src::Rec *__restrict__ recs_out)
{
    using Rec = typename Src::Rec;
    constexpr int kNb = 1 << kBits, kWaves = kThreads / 64;
    __shared__ uint32_t glob[kNb];         // next global position of each digit for this tile
    __shared__ uint16_t wc[kWaves][kNb];   // per wavefront of the current sub-tile: count of each digit
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned tile = xcd_tile();
    for (int d = tid; d < kNb; d += kThreads) {
        glob[d] = d < nd ? hist_off[(int64_t)d * gridDim.x + tile] : 0u;
#pragma unroll
        for (int w = 0; w < kWaves; w++) wc[w][d] = 0;
    }
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)tile * (kSub * kThreads);
    // clamped indexes (n > 0): every load in flight at once; the lanes
    // past the end take no part below
    uint32_t kv[kSub];
    Rec rv[kSub];
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const int64_t e = base + j * kThreads + tid;
        src.load(e < n ? e : n - 1, kv[j], rv[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSub; j++) {
        const bool valid = base + j * kThreads + tid < n;
        const uint32_t d = (src.sort_key(kv[j]) >> shift) & (kNb - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kBits; bit++) {
            const uint64_t m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        const uint32_t rk = (uint32_t)__popcll(peers & lt), cnt = (uint32_t)__popcll(peers);
        if (valid && rk == 0) wc[wv][d] = (uint16_t)cnt;
        __syncthreads();
        uint32_t before = 0, total = 0, pos = 0;
        if (valid) {
#pragma unroll
            for (int w = 0; w < kWaves; w++) {
                const uint32_t x = wc[w][d];
                before += w < wv ? x : 0u;
                total += x;
            }
            pos = glob[d] + before + rk;
        }
        __syncthreads();
        // every read of glob[] and wc[] of this sub-tile is done: the first
        // lane of each (wavefront, digit) clears its count, the one of the
        // last wavefront holding the digit advances the digit's position
        if (valid) {
            keys_out[pos] = kv[j];
            recs_out[pos] = rv[j];
            if (rk == 0) {
                wc[wv][d] = 0;
                if (before + cnt == total) glob[d] += total;
            }
        }
    }
}

// First sorted position of each bucket, from the bucket-ordered keys:
// bounds[s] is the first position whose bucket is >= s, for s in [0, n_bounds)
// (position n stands for the end).  Position p owns the buckets (bucket[p-1],
// bucket[p]] and writes p into each, so every entry is written once.
constexpr int64_t kShortRun = 16;
__global__ void __launch_bounds__(kBlock)
    k_slot_bounds(const uint32_t *__restrict__ keys, int64_t n, KeyDiv slot, uint32_t n_bounds,
                  uint32_t *__restrict__ bounds)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t lo = 1, hi = 0;
    if (p <= n) {
        lo = p == 0 ? 0 : (int64_t)slot(keys[p - 1]) + 1;
        hi = p == n ? (int64_t)n_bounds - 1 : (int64_t)slot(keys[p]);
    }
    const bool is_long = hi - lo + 1 > kShortRun;
    if (!is_long)
        for (int64_t c = lo; c <= hi; c++) bounds[c] = (uint32_t)p;
    uint64_t m = __ballot(is_long);
    const int lane = threadIdx.x & 63;
    while (m) {
        const int src = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int64_t l0 = __shfl(lo, src, 64), h0 = __shfl(hi, src, 64);
        const uint32_t v = (uint32_t)__shfl((int)p, src, 64);
        for (int64_t c = l0 + lane; c <= h0; c += 64) bounds[c] = v;
    }
}

// Exclusive scan over a workgroup of kThreads; *total receives the sum.
template <int kThreads>
__device__ __forceinline__ uint32_t block_excl_scan_n(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; w++) {
        off += (w < wid) ? wsum[w] : 0u;
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// Second phase: one workgroup per bucket orders the bucket's tracklets
// (in input order after the stable partition) by cell with a stable
// counting sort in LDS, over chunks of at most kCellChunk cells:
//  - count the tracklets of each cell of the chunk (LDS atomics);
//  - exclusive scan of the counts: the cells' offsets, written to `offsets`;
//  - per segment of kSeg tracklets, held in registers: a multisplit hands
//    wavefront w, in order, the tracklets whose cell c has c mod 8 = w; each
//    wavefront ranks its list 64 at a time (lanes with the same cell by
//    ballots, the first of them advancing the cell's cursor), so the eight
//    wavefronts rank disjoint cells at once; then every thread stores its
//    records at their places.
// Block n_slots (the number of buckets) copies the tracklets without a
// cell, still in input order, behind the valid ones and writes
// offsets[n_cells].
constexpr uint32_t kCellChunk = 16384;
constexpr int kCellBits = 14;                     // bits of a cell index within a chunk
constexpr int kOrderBlock = 512;                  // threads of the cell-order workgroup
constexpr int kOrderWaves = kOrderBlock / 64;     // = the number of cell classes
constexpr int kClassBits = 3;
constexpr int kOrderSub = 4;                      // tracklets per thread and segment
constexpr int kSeg = kOrderBlock * kOrderSub;     // tracklets per segment
constexpr uint32_t kNoSlot = 0xffffffffu;
constexpr int kClassEntries = kOrderWaves * kOrderSub * kOrderWaves;  // (class, sub-tile, wavefront)
static_assert(kOrderWaves == 1 << kClassBits, "one cell class per wavefront");
static_assert(kClassEntries <= kOrderBlock, "one scan entry per thread");
__device__ __forceinline__ int class_entry(int u, int w, int c) { return (u * kOrderWaves + w) * kOrderWaves + c; }

__global__ void __launch_bounds__(kOrderBlock)
    k_cell_order(const uint32_t *__restrict__ keys, const float4 *__restrict__ recs,
                 const uint32_t *__restrict__ bounds, int64_t bstride, int64_t n, uint32_t cells,
                 uint32_t chunk, uint32_t n_slots, float4 *__restrict__ sorted, uint32_t *__restrict__ offsets)
{
    extern __shared__ uint32_t lds[];
    uint32_t *cur = lds;                                          // [chunk] cell cursors
    uint32_t *sk = lds + chunk;                                   // [kSeg] cell, then slot
    uint16_t *lst = reinterpret_cast<uint16_t *>(lds + chunk + kSeg);  // [kSeg] tracklets by class
    __shared__ uint16_t ccnt[kClassEntries];  // per (sub-tile, wavefront, class): count, then offset
    __shared__ uint32_t cls_end[kOrderWaves];
    const uint32_t sl = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // bucket b starts at bounds[b * bstride]; the last one ends at n
    uint32_t end = sl < n_slots ? bounds[(int64_t)(sl + 1) * bstride] : (uint32_t)n;
    uint32_t start = bounds[(int64_t)sl * bstride];
    end = end > (uint64_t)n ? (uint32_t)n : end;
    start = start > end ? end : start;
    if (sl == n_slots) {
        for (uint32_t e = start + tid; e < end; e += kOrderBlock) sorted[e] = recs[e];
        if (tid == 0) offsets[(uint64_t)n_slots * cells] = start;
        return;
    }
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t done = start;
    for (uint32_t c0 = 0; c0 < cells; c0 += chunk) {
        const uint32_t cn = cells - c0 < chunk ? cells - c0 : chunk;
        const uint32_t kb = sl * cells + c0;  // key of the chunk's first cell
        for (uint32_t i = tid; i < cn; i += kOrderBlock) cur[i] = 0;
        __syncthreads();
        for (uint32_t b0 = start; b0 < end; b0 += kSeg) {
            // loads from a clamped index, all in flight at once (a guarded
            // load would wait for its data before the next one is issued)
            uint32_t lk[kOrderSub];
#pragma unroll
            for (int u = 0; u < kOrderSub; u++) {
                const uint32_t e = b0 + u * kOrderBlock + tid;
                lk[u] = keys[e < end ? e : end - 1];
            }
#pragma unroll
            for (int u = 0; u < kOrderSub; u++) {
                const uint32_t e = b0 + u * kOrderBlock + tid;
                lk[u] = e < end ? lk[u] - kb : cn;
            }
#pragma unroll
            for (int u = 0; u < kOrderSub; u++)
                if (lk[u] < cn) atomicAdd(&cur[lk[u]], 1u);
        }
        __syncthreads();
        // exclusive scan: thread t owns the cells [t * per, t * per + per)
        uint32_t chunk_total;
        {
            const uint32_t per = (cn + kOrderBlock - 1) / kOrderBlock;
            const uint32_t a = tid * per < cn ? tid * per : cn, b = a + per < cn ? a + per : cn;
            uint32_t sum = 0;
            for (uint32_t i = a; i < b; i++) sum += cur[i];
            uint32_t run = block_excl_scan_n<kOrderBlock>(sum, &chunk_total);
            for (uint32_t i = a; i < b; i++) {
                const uint32_t v = cur[i];
                cur[i] = run;
                run += v;
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < cn; i += kOrderBlock) offsets[kb + i] = done + cur[i];
        for (uint32_t s0 = start; s0 < end; s0 += kSeg) {
            // keys first, then records, from clamped indexes: the records
            // are still in flight while the keys are ranked
            uint32_t lk[kOrderSub], rk[kOrderSub];
            float4 rv[kOrderSub];
#pragma unroll
            for (int u = 0; u < kOrderSub; u++) {
                const uint32_t e = s0 + u * kOrderBlock + tid;
                lk[u] = keys[e < end ? e : end - 1];
            }
#pragma unroll
            for (int u = 0; u < kOrderSub; u++) {
                const uint32_t e = s0 + u * kOrderBlock + tid, k = lk[u] - kb;
                // (component-wise: a whole-struct copy put rv in scratch memory)
                const float4 r = recs[e < end ? e : end - 1];
                rv[u].x = r.x;
                rv[u].y = r.y;
                rv[u].z = r.z;
                rv[u].w = r.w;
                lk[u] = e < end && k < cn ? k : kNoSlot;
            }
            // multisplit by class: rank within the wavefront, count per (sub-tile, wavefront, class)
            if (tid < (uint32_t)kClassEntries) ccnt[tid] = 0;
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kOrderSub; u++) {
                const bool in = lk[u] != kNoSlot;
                const uint32_t c = lk[u] & (kOrderWaves - 1);
                sk[u * kOrderBlock + tid] = lk[u];
                uint64_t peers = __ballot(in);
#pragma unroll
                for (int bit = 0; bit < kClassBits; bit++) {
                    const uint64_t bm = __ballot((c >> bit) & 1u);
                    peers &= ((c >> bit) & 1u) ? bm : ~bm;
                }
                rk[u] = (uint32_t)__popcll(peers & lt);
                if (in && rk[u] == 0) ccnt[class_entry(u, wv, c)] = (uint16_t)__popcll(peers);
            }
            __syncthreads();
            // exclusive offsets in (class, sub-tile, wavefront) order: thread t
            // holds the t-th entry of that order
            {
                constexpr int kPerClass = kOrderSub * kOrderWaves;
                const int c = (int)tid / kPerClass, u = ((int)tid / kOrderWaves) % kOrderSub,
                          w = (int)tid % kOrderWaves;
                const bool has = tid < (uint32_t)kClassEntries;
                const uint32_t v = has ? ccnt[class_entry(u, w, c)] : 0u;
                uint32_t tot;
                const uint32_t off = block_excl_scan_n<kOrderBlock>(v, &tot);
                if (has) {
                    ccnt[class_entry(u, w, c)] = (uint16_t)off;
                    if ((int)tid % kPerClass == kPerClass - 1) cls_end[c] = off + v;
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kOrderSub; u++)
                if (lk[u] != kNoSlot)
                    lst[ccnt[class_entry(u, wv, lk[u] & (kOrderWaves - 1))] + rk[u]] =
                        (uint16_t)(u * kOrderBlock + tid);
            __syncthreads();
            // wavefront wv ranks the tracklets of class wv in order
            const uint32_t l0 = wv == 0 ? 0u : cls_end[wv - 1], l1 = cls_end[wv];
            for (uint32_t j0 = l0; j0 < l1; j0 += 64) {
                const uint32_t j = j0 + lane;
                const bool ok = j < l1;
                const uint32_t i = ok ? lst[j] : 0u;
                const uint32_t c = ok ? sk[i] : 0u;
                uint64_t peers = __ballot(ok);
#pragma unroll
                for (int bit = kClassBits; bit < kCellBits; bit++) {
                    const uint64_t bm = __ballot((c >> bit) & 1u);
                    peers &= ((c >> bit) & 1u) ? bm : ~bm;
                }
                const uint32_t r = (uint32_t)__popcll(peers & lt);
                const uint32_t slot = ok ? cur[c] + r : 0u;
                wave_sync();
                if (ok && r == 0) cur[c] = slot + (uint32_t)__popcll(peers);
                if (ok) sk[i] = slot;
                wave_sync();
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kOrderSub; u++)
                if (lk[u] != kNoSlot) sorted[done + sk[u * kOrderBlock + tid]] = rv[u];
            __syncthreads();
        }
        done += chunk_total;
    }
}

// load the N values owned by this thread (pad past the end)
template <int N>
__device__ __forceinline__ void load_items(const uint32_t *in, int64_t n, int64_t base, uint32_t pad,
                                           uint32_t (&v)[N])
{
    if (base + N <= n) {
        const uint4 *q = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int j = 0; j < N / 4; j++) {
            const uint4 u = q[j];
            v[4 * j] = u.x;
            v[4 * j + 1] = u.y;
            v[4 * j + 2] = u.z;
            v[4 * j + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; j++) v[j] = (base + j < n) ? in[base + j] : pad;
    }
}

// store the N values owned by this thread (nothing past the end)
template <int N>
__device__ __forceinline__ void store_items(uint32_t *out, int64_t n, int64_t base, const uint32_t (&v)[N])
{
    if (base + N <= n) {
        uint4 *q = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int j = 0; j < N / 4; j++)
            q[j] = make_uint4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < N; j++)
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
static int64_t wide_blocks(int64_t n, int threads) { return (n + kSub * threads - 1) / (kSub * threads); }
int64_t tkl_hist_len(int64_t n) { return radix_blocks(n > 0 ? n : 1) * (int64_t)(1 << kWideBits); }

// exclusive sum scan of n values (out may alias nothing of in)
static void launch_excl_scan(const uint32_t *in, int64_t n, uint32_t *tiles, uint32_t *out,
                             hipStream_t s)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) return;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tiles);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tiles, out);
}

// One 8-bit radix pass from src into (keys_out, recs_out).
template <typename Src>
static void radix_pass(const Src &src, int64_t n, int shift, uint32_t *hist, uint32_t *hist_off,
                       uint32_t *tiles, uint32_t *keys_out, typename Src::Rec *recs_out, hipStream_t s,
                       uint32_t *rank_out = nullptr)
{
    const int64_t nblk = radix_blocks(n);
    hipLaunchKernelGGL((k_radix_hist<Src, kRadixBits>), dim3((unsigned)nblk), dim3(kBlock), 0, s, src, n, shift,
                       kBins, hist, (uint32_t *)nullptr);
    launch_excl_scan(hist, nblk * kBins, tiles, hist_off, s);
    hipLaunchKernelGGL(k_radix_scatter<Src>, dim3((unsigned)nblk), dim3(kBlock), 0, s, src, n, shift, hist,
                       hist_off, keys_out, recs_out, rank_out);
}

// First pass of the tracklet partition, over the low kBits of the bucket:
// the histogram pass computes the keys once and leaves them in key_cache for
// the scatter.
template <int kBits, typename Src>
static void wide_pass_tkl(Src src, int64_t n, int nd, uint32_t *key_cache, uint32_t *hist, uint32_t *hist_off,
                          uint32_t *tiles, uint32_t *keys_out, float4 *recs_out, hipStream_t s)
{
    constexpr int kT = kWideThreads<kBits>;
    const int64_t nblk = wide_blocks(n, kT);
    src.cached = nullptr;
    hipLaunchKernelGGL((k_radix_hist<Src, kBits, kT>), dim3((unsigned)nblk), dim3(kT), 0, s, src, n, 0, nd, hist,
                       key_cache);
    launch_excl_scan(hist, nblk * nd, tiles, hist_off, s);
    src.cached = key_cache;
    hipLaunchKernelGGL((k_wide_scatter<Src, kBits, kT>), dim3((unsigned)nblk), dim3(kT), 0, s, src, n, 0, nd,
                       hist_off, keys_out, recs_out);
}

template <typename Src>
static void first_pass_tkl(const Src &src, int wide, int64_t n, int nd, uint32_t *key_cache, const BinBuffers &buf,
                           uint32_t *keys_out, float4 *recs_out, hipStream_t s)
{
    if (wide == 10)
        wide_pass_tkl<10>(src, n, nd, key_cache, buf.hist, buf.hist_off, buf.tiles_tkl, keys_out, recs_out, s);
    else
        wide_pass_tkl<kWideBits>(src, n, nd, key_cache, buf.hist, buf.hist_off, buf.tiles_tkl, keys_out, recs_out, s);
}

static int bit_length(uint64_t v)
{
    int bits = 1;
    while (bits < 64 && v >> bits) bits++;
    return bits;
}

static int radix_passes(uint64_t max_key) { return (bit_length(max_key) + kRadixBits - 1) / kRadixBits; }

void launch_bin(const float *y, const float *z, const float *dy, const uint32_t *det_row,
                const int32_t *grp, int64_t n, const BinCfg &b, BinBuffers &buf, hipStream_t s)
{
    // Buckets of g consecutive chamber slots (g divides 540): the fewest
    // slots per bucket that keep the partition to one pass, as long as a
    // bucket's cells fit one LDS chunk of the cell order (small slots are
    // thus merged into buckets of useful size for one workgroup).
    const uint32_t per_slot = (uint32_t)b.n_db * (uint32_t)b.n_yb * (uint32_t)b.n_rows;
    const uint32_t n_chambers = (uint32_t)b.n_groups * (uint32_t)kDet;
    static const uint32_t kDivisors[] = {1, 2, 3, 4, 5, 6, 9, 10, 12, 15, 18, 20, 27, 30, 36, 45, 54, 60,
                                         90, 108, 135, 180, 270, 540};
    uint32_t g = 1;
    for (uint32_t d : kDivisors) {
        if ((uint64_t)d * per_slot > kCellChunk) break;
        g = d;
        if (n_chambers / d + 1 <= (1u << kWideBits)) break;
    }
    const uint32_t cells = g * per_slot;        // per bucket
    const uint32_t n_slots = n_chambers / g;    // buckets
    const KeyDiv slot{cells, 1.0 / (double)cells};
    // buckets 0 .. n_slots (the last: tracklets without a cell)
    const int bits = bit_length(n_slots);
    const int wide = bits <= 10 ? 10 : kWideBits;
    const int passes = 1 + (bits > wide ? (bits - wide + kRadixBits - 1) / kRadixBits : 0);
    // ping-pong so that the last pass lands in recs_tmp, the cell order's input
    uint32_t *kdst[2] = {buf.keys_a, buf.keys_b};
    float4 *rdst[2] = {buf.recs_tmp, buf.sorted};
    int out = (passes - 1) & 1;
    // digits of the first pass that occur: every bucket of a one-pass partition
    const int nd = passes == 1 ? (int)n_slots + 1 : 1 << wide;
    if (n > 0) {
        // the other key buffer is free during the first pass
        if (grp)
            first_pass_tkl(TklSrc<true>{y, z, dy, det_row, grp, b, slot, nullptr}, wide, n, nd, kdst[out ^ 1], buf,
                           kdst[out], rdst[out], s);
        else
            first_pass_tkl(TklSrc<false>{y, z, dy, det_row, nullptr, b, slot, nullptr}, wide, n, nd, kdst[out ^ 1],
                           buf, kdst[out], rdst[out], s);
        for (int p = 1; p < passes; p++) {
            const SlotPassSrc ps{kdst[out], rdst[out], slot};
            out ^= 1;
            radix_pass(ps, n, wide + (p - 1) * kRadixBits, buf.hist, buf.hist_off, buf.tiles_tkl, kdst[out],
                       rdst[out], s);
        }
    }
    // out == 0 here: keys_a and recs_tmp hold the tracklets in bucket order.
    // After a one-pass partition, bucket b starts where its digit starts for
    // the first tile (hist_off[b * tiles]); otherwise the starts are found
    // from the partitioned keys.
    const uint32_t *bnd = buf.hist_off;
    int64_t bstride = wide_blocks(n, wide == 10 ? kWideThreads<10> : kWideThreads<kWideBits>);
    if (n == 0 || passes > 1) {
        hipLaunchKernelGGL(k_slot_bounds, dim3(grid_for(n + 1, kBlock)), dim3(kBlock), 0, s, buf.keys_a, n, slot,
                           n_slots + 2, buf.bstart);
        bnd = buf.bstart;
        bstride = 1;
    }
    const uint32_t chunk = cells < kCellChunk ? cells : kCellChunk;
    const size_t lds = (chunk + kSeg) * sizeof(uint32_t) + kSeg * sizeof(uint16_t);
    if (lds > 65536)  // up to 88 KB for a full chunk
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cell_order),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_cell_order, dim3(n_slots + 1), dim3(kOrderBlock), lds, s, buf.keys_a, buf.recs_tmp, bnd,
                       bstride, n, cells, chunk, n_slots, buf.sorted, buf.offsets);
}

template <typename TS>
static void track_sort(const TS *ip, const int32_t *isec, const int32_t *igrp, int64_t n, int32_t n_groups,
                       const TrackOrder &o, hipStream_t s)
{
    const int passes = radix_passes((uint64_t)(n_groups * kSectors) << kOrderPosBits);
    uint32_t *kb[2] = {o.key_a, o.key_b};
    uint32_t *vb[2] = {o.val_a, o.val_b};
    if (igrp)
        radix_pass(TrkSrc<TS, true>{ip, isec, igrp, n, n_groups}, n, 0, o.hist, o.hist_off, o.tiles, kb[0], vb[0],
                   s, passes == 1 ? o.rank : nullptr);
    else
        radix_pass(TrkSrc<TS, false>{ip, isec, nullptr, n, n_groups}, n, 0, o.hist, o.hist_off, o.tiles, kb[0],
                   vb[0], s, passes == 1 ? o.rank : nullptr);
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
