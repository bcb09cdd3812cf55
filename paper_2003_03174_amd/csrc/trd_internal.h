// Internal declarations shared by the HIP translation units of libtrd.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trd {

constexpr int kLayers = 6;
constexpr int kSectors = 18;
constexpr int kStacks = 5;
constexpr int kDet = 540;

// per-track status bits (same values as TRD_TRK_* of the public header)
constexpr uint32_t kStopSnp = 1u, kRotFail = 2u, kOutOfZ = 4u, kFallback = 8u, kNotPD = 16u,
                   kBadInput = 32u, kRefitFew = 64u, kRefitSkip = 128u, kStopped = 256u;
constexpr int kAbsentWords = (kDet + 31) / 32;

// Cell geometry of the tracklet binning; the key arithmetic runs in double
// so that floor() sees the exact difference y - y_min (w is a power of two).
struct BinCfg {
    double y_min;   // -w * n_yb / 2
    double inv_w;   // 1 / w, exact
    double dy_min;  // same for the deflection bins
    double inv_wd;
    int32_t n_rows, n_yb, n_db, n_groups;
    uint32_t n_cells;
    uint32_t absent[kAbsentWords];  // bit d: chamber slot d has no chamber
};

__host__ __device__ inline bool slot_absent(const BinCfg &b, int det)
{
    return (b.absent[det >> 5] >> (det & 31)) & 1u;
}

// Matching parameters, converted once to the state precision T.
template <typename T>
struct DevCfg {
    T x_layer[kLayers];
    T tilt[kLayers];
    T z_min, z_max, pad_len, inv_pad, vz;  // vz = pad_len^2 / 12
    T drift_len, k_curv;                   // k_curv = -kappa * Bz
    T x_over_x0, mass2;
    // energy loss: eloss_xrho (g/cm^2, 0 = off), K Z/A, 1/I^2, m, m_e/m
    T eloss_xrho, eloss_kza, inv_i2, mass, me_over_m;
    T sigma_y[3], sigma_dy[3], tan_psi;
    T chi2_max, n_sigma_dy, n_sigma_road, snp_max;
    T chi2_penalty;                            // cost of a layer without a tracklet (hypotheses)
    T tan_half_sector, cos_sector, sin_sector;  // tan(10 deg), cos/sin(20 deg)
    T dx_max;
    const T *dx;                               // [540] device
    // field map: Bz = bz (1 + fr (x^2 + y^2) + fz z^2) in any sector frame
    int field_on;
    T fr, fz;
    double field_step;                         // largest integration step (cm)
    BinCfg bin;
};

// Device buffers of the binning.
struct BinBuffers {
    uint32_t *keys_a, *keys_b;  // [cap] cell keys (partition ping-pong)
    float4 *sorted, *recs_tmp;  // [cap] records (partition ping-pong; result in `sorted`)
    uint32_t *hist, *hist_off;  // [tkl_hist_len(cap)] digit histograms
    uint32_t *tiles_tkl;        // [scan_block_sums_len(tkl_hist_len(cap))]
    uint32_t *offsets;          // [n_cells + 1]
    uint32_t *bstart;           // [n_groups * kDet + 2] first position of each bucket
};

// launchers (stream-ordered, no synchronisation)
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
int64_t scan_block_sums_len(int64_t n);
int64_t radix_blocks(int64_t n);
int64_t tkl_hist_len(int64_t n);  // histogram entries of the tracklet partition of n
// sorts the tracklets into cells: buf.sorted in (key, input index) order,
// buf.offsets[c] = first position of cell c, offsets[n_cells] = valid count;
// the tracklets without a cell follow in input order
void launch_bin(const float *y, const float *z, const float *dy, const uint32_t *det_row,
                const int32_t *grp, int64_t n, const BinCfg &b, BinBuffers &buf, hipStream_t s);

struct MatchIO {
    const float4 *sorted;
    const uint32_t *offsets;
    const void *ip, *ic, *ix;
    const int32_t *isec, *igrp;
    int64_t n;
    int32_t *oidx;
    void *op, *oc, *ox;
    int32_t *osec;
    void *ochi2, *ochi2l;
    int32_t *onm;
    uint32_t *ost;
    int32_t *fb_list;    // FP32 mode: tracks to re-run with a double covariance
    uint32_t *fb_count;  // [1]
    uint32_t *fb_done;   // [1]
    int force_fallback;  // test hook: queue every track for the re-run
    uint32_t *work_next; // [1] persistent launch: next block of tracks
    uint32_t *work_done; // [1] persistent launch: finished workgroups
    // Ordered mode (both set): track i of the launch is row i of rows_in and
    // its results go to row i of rows_out, instead of the caller's arrays.
    const void *rows_in;  // [n][kRowIn] of the state type
    void *rows_out;       // [n][kRowOut] of the state type
    int row_out;  // entries per result row: kRowOut, or kRowOutShort without chi2 per layer
    // host side only: events that take the main match kernel's start and end
    // (or null)
    hipEvent_t ev_begin, ev_end;
};

// Launch of the main match kernel.  With the caller's events the dispatch
// itself stamps them at the kernel's start and end, in place of an event
// record on each side (which left longer gaps around the kernel); a stream
// under graph capture records them around the kernel instead (event nodes).
template <typename K, typename... A>
inline void launch_timed(const MatchIO &io, K kernel, dim3 grid, dim3 block, hipStream_t s, A... args)
{
    if (io.ev_begin) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cap) != hipSuccess) {
            (void)hipGetLastError();  // a refused query leaves no error for the call to report
            cap = hipStreamCaptureStatusActive;
        }
        if (cap == hipStreamCaptureStatusNone) {
            hipExtLaunchKernelGGL(kernel, grid, block, 0u, s, io.ev_begin, io.ev_end, 0u, args...);
            return;
        }
    }
    if (io.ev_begin) (void)hipEventRecord(io.ev_begin, s);
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    if (io.ev_end) (void)hipEventRecord(io.ev_end, s);
}

// Rows of the ordered mode, in units of the state type.
// in:  p[5], cov[15], x, sector, group (integers stored bit-exact), pad
// out: p[5], cov[15], x, chi2, sector, n_match, status, idx[6], pad, chi2[6], pad
constexpr int kRowIn = 24;
constexpr int kRowOut = 40;
constexpr int kRowOutShort = 32;  // without the chi2 per layer
constexpr int kRowChi2 = 32;      // first chi2-per-layer entry of a long row
// the order key holds the group and sector above 11 position bits
constexpr int kOrderPosBits = 11;
constexpr int32_t kMaxOrderGroups = (1 << (32 - kOrderPosBits)) / kSectors;

// TRD-only refit: inputs and outputs (device arrays of the state type where
// untyped; see trd_refit in the public header).
struct RefitIO {
    const void *ip, *ix;
    const int32_t *isec, *idx;
    const float *y, *z;
    const uint32_t *det_row;
    int64_t n, n_tkl;
    double cov0[5];
    int32_t min_tracklets;
    void *op, *oc, *ox, *ochi2;
    int32_t *osec, *onused;
    uint32_t *ost;
};
void launch_refit(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf, const RefitIO &io,
                  hipStream_t s);

// Residual maps: reference tracks, TPC clusters, voxel sums (see
// trd_residual_sums in the public header).
constexpr int kVoxelSums = 8;
constexpr int kMaxVoxels = 2048;  // the per-workgroup LDS copy of the sums: 64 KB (float), 128 KB (double)
struct ResidualIO {
    const void *rp, *rx;
    const int32_t *rsec;
    const uint32_t *rstatus;
    const float *cy, *cz;
    const uint32_t *row_sec;
    const int64_t *first;
    int64_t n;
    double *sums;
    double x_in, x_out;
    int32_t n_rows, nx, ny, nz, nvox;
};
void launch_residual_sums(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf,
                          const ResidualIO &io, int n_cu, hipStream_t s);
void launch_voxel_solve(const double *sums, int nvox, int min_count, float *dist, hipStream_t s);

// Processing-order key of a seed: group and sector, then a class of |q/pT|
// (road widths grow with the scattering of slow tracks, so a wavefront of
// similar tracks diverges less), then 32 cm in z and 8 cm in y (clamped);
// rejected seeds get the largest key.
template <typename TS>
__device__ __forceinline__ uint32_t track_order_key(TS y, TS z, TS c, int sec, int grp, int32_t n_groups)
{
    // without branches, so that the loads of several seeds can be in flight
    // at once (the bins of a seed that is not valid are computed and dropped)
    const bool ok = (sec >= 0) & (sec < kSectors) & (grp >= 0) & (grp < n_groups) & __builtin_isfinite(y) &
                    __builtin_isfinite(z);
    const TS zs = (z + TS(512)) * TS(0.03125), ys = (y + TS(64)) * TS(0.125);
    const uint32_t zb = (uint32_t)(int)fmin(fmax(zs, TS(0)), TS(31));
    const uint32_t yb = (uint32_t)(int)fmin(fmax(ys, TS(0)), TS(15));
    const TS ac = fabs(c);
    const uint32_t pb = (uint32_t)!(ac < TS(0.8)) + (uint32_t)!(ac < TS(1.6)) + (uint32_t)!(ac < TS(2.5));
    const uint32_t k = ((uint32_t)(grp * kSectors + sec) << kOrderPosBits) | (pb << 9) | (zb << 4) | yb;
    const uint32_t m = 0u - (uint32_t)ok;
    return (k & m) | (((uint32_t)(n_groups * kSectors) << kOrderPosBits) & ~m);
}

// buffers of the spatial track order (capacity n each unless noted)
struct TrackOrder {
    uint32_t *key_a, *key_b, *val_a, *val_b;  // sort ping-pong
    uint32_t *rank;                           // rank[i]: row of input track i
    uint32_t *hist, *hist_off, *tiles;        // radix_blocks(n) * 256, its scan tiles
    void *rows_in, *rows_out;
};

// Stable sort of the seeds by track_order_key (state of type double for
// precision 0, float otherwise, p component-major as in the C ABI); fills
// o.rank.  Overwrites key_a/b, val_a/b, hist, hist_off, tiles.
void launch_track_sort(int precision, const void *ip, const int32_t *isec, const int32_t *igrp, int64_t n,
                       int32_t n_groups, const TrackOrder &o, hipStream_t s);

// Sorts the tracks by (group, sector, z, y) of the seed, packs their state
// into io.rows_in in that order and points io at the rows.
void launch_order_in(int precision, MatchIO &io, int32_t n_groups, const TrackOrder &o, hipStream_t s);
// Copies the result rows back to the caller's arrays in input order.
void launch_order_out(int precision, const MatchIO &io, const TrackOrder &o, hipStream_t s);

// precision: 0 = FP64, 1 = FP32 (+ fallback), 2 = FP32 state / FP64 covariance
// lanes: lanes that scan one track's road together (1 = one lane per track)
// several hypotheses per track: n_hyp lanes per track (1, 2, 4 or 8)
void launch_beam(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf, const MatchIO &io,
                 int n_hyp, hipStream_t s);
// persistent: one resident grid pulling blocks of tracks (lanes == 1 only)
void launch_match(int precision, const DevCfg<double> &gd, const DevCfg<float> &gf,
                  const MatchIO &io, int block, int lanes, bool persistent, int n_cu, hipStream_t s);

}  // namespace trd
