// Host side of the C ABI (include/trd.h): configuration checks, the
// context's device buffers, and the stream-ordered launch sequences of
// trd_load_tracklets and trd_match.  Nothing here synchronises the stream
// except trd_reserve/trd_destroy (allocation, free).
#include <math.h>
#include <mutex>
#include <new>
#include <string.h>

#include "../../include/trd.h"
#include "trd_internal.h"

using namespace trd;

struct trd_ctx {
    int device = 0;
    trd_config cfg{};
    DevCfg<double> gd{};
    DevCfg<float> gf{};
    double *d_dx64 = nullptr;
    float *d_dx32 = nullptr;
    uint32_t *d_small = nullptr;  // [0] fb_count [1] fb_done [2] work_next [3] work_done
    int n_cu = 0;

    // tracklet-side capacity
    int64_t cap_tkl = 0;
    uint32_t *d_keys_a = nullptr, *d_keys_b = nullptr;
    float4 *d_sorted = nullptr, *d_tmp = nullptr;
    uint32_t *d_hist = nullptr, *d_hist_off = nullptr, *d_tiles_tkl = nullptr;
    // cell-side capacity (entries of offsets minus one)
    int64_t cap_cells = 0;
    uint32_t *d_offsets = nullptr;
    // track-side capacity
    int64_t cap_trk = 0;
    int32_t *d_fb = nullptr;
    // processing order of the tracks (spatial sort) and the state rows in it
    uint32_t *d_tkey_a = nullptr, *d_tkey_b = nullptr, *d_tval_a = nullptr, *d_tval_b = nullptr;
    uint32_t *d_trank = nullptr, *d_thist = nullptr, *d_thist_off = nullptr, *d_ttiles = nullptr;
    unsigned char *d_rows_in = nullptr, *d_rows_out = nullptr;

    // trd_load_and_match: a stream of the context (default priority) that runs
    // the seeds' ordering beside the binning, and the events of its fork and join
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;

    // TRD_CFG_TIME_KERNEL: a ring of event pairs around the main match kernel
    static constexpr int kEvRing = 64;
    hipEvent_t ev[kEvRing][2] = {};
    int64_t ev_count = 0;

    int64_t bytes = 0;
    bool loaded = false;
    int64_t n_tkl = 0;
    int32_t n_groups = 0;
    int64_t n_cells = 0;
};

namespace {

// ---- scratch of trd_match_noalloc -----------------------------------------
// One file-scope device array per GPU (each device holds its own copy while
// the library is loaded): the float path's re-run queue and the four
// counters of the match kernels.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in); trd_create takes its device
// address once per device with hipGetSymbolAddress and every later use goes
// through that address.
constexpr int64_t kNoAllocMaxTracks = int64_t(1) << 21;  // 8 MB of queue
constexpr int64_t kScratchHead = 64;                    // counters, padded to 256 bytes
static __device__ __align__(256) uint32_t scratch[kScratchHead + kNoAllocMaxTracks];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxScratchDevices] = {};

// Takes the device address of `scratch` on the current device `dev` once.
int scratch_setup(int dev)
{
    if (dev >= kMaxScratchDevices) return TRD_OK;  // trd_match_noalloc then refuses this device
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return TRD_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return TRD_EDEVICE;
    }
    g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
    return TRD_OK;
}

uint32_t *scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

bool finite_all(const double *v, int n)
{
    for (int i = 0; i < n; i++)
        if (!isfinite(v[i])) return false;
    return true;
}

int check_config(const trd_config *c)
{
    if (!c || c->struct_size != sizeof(trd_config)) return TRD_EINVAL;
    if (c->precision < TRD_PREC_FP64 || c->precision > TRD_PREC_FP32_COV64) return TRD_EINVAL;
    if (c->n_rows < 1 || c->n_rows > 32 || c->n_yb < 1 || c->n_yb > 4096) return TRD_EINVAL;
    if (c->n_db < 1 || c->n_db > 4096) return TRD_EINVAL;
    int ex;
    for (double wb : {c->y_bin_w, c->dy_bin_w})
        if (!(wb > 0) || !isfinite(wb) || frexp(wb, &ex) != 0.5) return TRD_EINVAL;  // power of two
    if (!finite_all(c->x_layer, 6) || !finite_all(c->tilt, 6) || !finite_all(c->dx_chamber, 540))
        return TRD_EINVAL;
    for (int l = 0; l < 6; l++)
        if (!(c->x_layer[l] > 0)) return TRD_EINVAL;
    const double sc[] = {c->z_min, c->pad_len, c->drift_len, c->bz, c->x_over_x0, c->mass,
                         c->tan_psi, c->chi2_max, c->n_sigma_dy, c->n_sigma_road, c->snp_max};
    if (!finite_all(sc, 11) || !finite_all(c->sigma_y, 3) || !finite_all(c->sigma_dy, 3))
        return TRD_EINVAL;
    if (!(c->pad_len > 0) || !(c->z_min < 0) || !(c->snp_max > 0 && c->snp_max <= 1) ||
        !(c->n_sigma_road > 0) || !(c->n_sigma_dy > 0) || !(c->chi2_max > 0) || c->x_over_x0 < 0)
        return TRD_EINVAL;
    // the stacks' pad rows tile [z_min, -z_min]
    if (fabs(2 * c->z_min + TRD_N_STACKS * c->n_rows * c->pad_len) > 1e-9 * fabs(c->z_min))
        return TRD_EINVAL;
    if (c->block_size != 0 && (c->block_size < 64 || c->block_size > 256 || c->block_size % 64))
        return TRD_EINVAL;
    switch (c->search_lanes) {
    case 0: case 1: case 4: case 8: case 16: case 32: case 64: break;
    default: return TRD_EINVAL;
    }
    // the persistent grid is a one-lane-per-track schedule
    if ((c->flags & TRD_CFG_PERSISTENT) && c->search_lanes > 1) return TRD_EINVAL;
    switch (c->n_hyp) {
    case 0: case 1: case 2: case 4: case 8: break;
    default: return TRD_EINVAL;
    }
    if (c->n_hyp > 0 && (c->search_lanes > 1 || (c->flags & TRD_CFG_PERSISTENT))) return TRD_EINVAL;
    if (c->n_hyp > 0 && !(c->chi2_penalty >= 0 && c->chi2_penalty < 1e30)) return TRD_EINVAL;
    for (int k = 0; k < 5; k++)
        if (!(c->refit_cov[k] > 0 && c->refit_cov[k] < 1e30)) return TRD_EINVAL;
    if (c->refit_min < 1 || c->refit_min > 6) return TRD_EINVAL;
    if (!(c->tpc_x_in > 0 && c->tpc_x_out > c->tpc_x_in && c->tpc_x_out < 1e4) || c->tpc_n_rows < 2 ||
        c->tpc_n_rows > 65535 || c->vox_nx < 1 || c->vox_ny < 1 || c->vox_nz < 1 || c->vox_min < 1)
        return TRD_EINVAL;
    if ((int64_t)TRD_N_SECTORS * c->vox_nx * c->vox_ny * c->vox_nz > kMaxVoxels) return TRD_EINVAL;
    if (!(c->eloss_xrho >= 0 && c->eloss_xrho < 1e6)) return TRD_EINVAL;
    if (!(fabs(c->field_br) < 1 && fabs(c->field_bz) < 1)) return TRD_EINVAL;
    if ((c->field_br != 0 || c->field_bz != 0) && !(c->field_step > 0 && c->field_step <= 20)) return TRD_EINVAL;
    if (c->eloss_xrho > 0 && !(c->eloss_za > 0 && c->eloss_za < 2 && c->eloss_i > 0 && c->eloss_i < 1 &&
                               c->mass > 0 && isfinite(c->eloss_i)))
        return TRD_EINVAL;
    return TRD_OK;
}

template <typename T>
void fill_devcfg(DevCfg<T> &g, const trd_config &c, const T *dx)
{
    for (int l = 0; l < 6; l++) {
        g.x_layer[l] = (T)c.x_layer[l];
        g.tilt[l] = (T)c.tilt[l];
    }
    g.z_min = (T)c.z_min;
    g.z_max = (T)(-c.z_min);
    g.pad_len = (T)c.pad_len;
    g.inv_pad = (T)(1.0 / c.pad_len);
    g.vz = (T)(c.pad_len * c.pad_len / 12.0);
    g.drift_len = (T)c.drift_len;
    g.k_curv = (T)(-2.99792458e-3 * c.bz);
    g.x_over_x0 = (T)c.x_over_x0;
    g.mass2 = (T)(c.mass * c.mass);
    g.eloss_xrho = (T)c.eloss_xrho;
    g.eloss_kza = (T)(0.307075e-3 * c.eloss_za);
    g.inv_i2 = c.eloss_xrho > 0 ? (T)(1.0 / (c.eloss_i * c.eloss_i)) : (T)0;
    g.mass = (T)c.mass;
    g.me_over_m = c.mass > 0 ? (T)(0.51099895e-3 / c.mass) : (T)0;
    for (int k = 0; k < 3; k++) {
        g.sigma_y[k] = (T)c.sigma_y[k];
        g.sigma_dy[k] = (T)c.sigma_dy[k];
    }
    g.tan_psi = (T)c.tan_psi;
    g.chi2_max = (T)c.chi2_max;
    g.n_sigma_dy = (T)c.n_sigma_dy;
    g.n_sigma_road = (T)c.n_sigma_road;
    g.snp_max = (T)c.snp_max;
    g.chi2_penalty = (T)c.chi2_penalty;
    const double dphi = 2.0 * M_PI / TRD_N_SECTORS;
    g.tan_half_sector = (T)tan(0.5 * dphi);
    g.cos_sector = (T)cos(dphi);
    g.sin_sector = (T)sin(dphi);
    double dxm = 0;
    for (int d = 0; d < TRD_N_DET; d++) dxm = fmax(dxm, fabs(c.dx_chamber[d]));
    g.dx_max = (T)dxm;
    g.dx = dx;
    g.field_on = (c.field_br != 0 || c.field_bz != 0) ? 1 : 0;
    g.fr = (T)(c.field_br / (370.0 * 370.0));
    g.fz = (T)(c.field_bz / (360.0 * 360.0));
    g.field_step = c.field_step;
    g.bin.y_min = -c.y_bin_w * c.n_yb / 2.0;
    g.bin.inv_w = 1.0 / c.y_bin_w;
    g.bin.dy_min = -c.dy_bin_w * c.n_db / 2.0;
    g.bin.inv_wd = 1.0 / c.dy_bin_w;
    g.bin.n_rows = c.n_rows;
    g.bin.n_yb = c.n_yb;
    g.bin.n_db = c.n_db;
    g.bin.n_groups = 1;
    g.bin.n_cells = 0;
    for (int w = 0; w < kAbsentWords; w++) g.bin.absent[w] = 0;
    for (int d = 0; d < TRD_N_DET; d++)
        if (c.chamber_absent[d]) g.bin.absent[d >> 5] |= 1u << (d & 31);
}

int hip_status(hipError_t e) { return e == hipSuccess ? TRD_OK : TRD_EDEVICE; }

template <typename T>
int dev_alloc(trd_ctx *ctx, T **p, int64_t count, int64_t *bytes_acc)
{
    const size_t sz = sizeof(T) * (size_t)(count > 0 ? count : 1);
    void *q = nullptr;
    if (hipMalloc(&q, sz) != hipSuccess) {
        (void)hipGetLastError();
        return TRD_ENOMEM;
    }
    *p = static_cast<T *>(q);
    *bytes_acc += (int64_t)sz;
    (void)ctx;
    return TRD_OK;
}

template <typename T> void dev_free(T **p)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

int64_t hist_len(int64_t n) { return radix_blocks(n > 0 ? n : 1) * 256; }
int64_t tkl_bytes(int64_t n)
{
    const int64_t m = n > 0 ? n : 1;
    return m * (4 + 4 + 16 + 16) + 8 * tkl_hist_len(n) + 4 * scan_block_sums_len(tkl_hist_len(n));
}
// chamber slots of nc cells (cells per slot: n_rows * n_db * n_yb)
int64_t n_slots_of(const trd_config &c, int64_t nc) { return nc / ((int64_t)c.n_rows * c.n_db * c.n_yb); }
// offsets [nc + 1], then the first position of each slot [slots + 2]
int64_t cell_entries(const trd_config &c, int64_t nc) { return nc + 1 + n_slots_of(c, nc) + 2; }
int64_t cell_bytes(const trd_config &c, int64_t nc) { return 4 * cell_entries(c, nc); }
// tracks are matched in a spatial order (rows of state in, rows of results
// out) unless the caller keeps its own order or the launch shape has no use
// for it (several lanes per road)
bool ordered(const trd_config &c)
{
    return !(c.flags & TRD_CFG_INPUT_ORDER) && c.search_lanes <= 1;
}
int64_t row_scalar(const trd_config &c) { return c.precision == TRD_PREC_FP64 ? 8 : 4; }
int64_t trk_bytes(const trd_config &c, int64_t n)
{
    const int64_t m = n > 0 ? n : 1;
    int64_t b = 4 * m;
    if (ordered(c))
        b += m * (20 + (kRowIn + kRowOut) * row_scalar(c)) + 8 * hist_len(m) +
             4 * scan_block_sums_len(hist_len(m));
    return b;
}

int over_budget(const trd_ctx *ctx, int64_t extra)
{
    const uint64_t b = ctx->cfg.hbm_budget_bytes;
    return b != 0 && (uint64_t)(ctx->bytes + extra) > b;
}

void free_tkl(trd_ctx *ctx)
{
    dev_free(&ctx->d_keys_a);
    dev_free(&ctx->d_keys_b);
    dev_free(&ctx->d_sorted);
    dev_free(&ctx->d_tmp);
    dev_free(&ctx->d_hist);
    dev_free(&ctx->d_hist_off);
    dev_free(&ctx->d_tiles_tkl);
}

int ensure_tkl(trd_ctx *ctx, int64_t n)
{
    if (n <= ctx->cap_tkl && ctx->d_keys_a) return TRD_OK;
    int64_t cap = n > 2 * ctx->cap_tkl ? n : 2 * ctx->cap_tkl;
    const int64_t old = ctx->d_keys_a ? tkl_bytes(ctx->cap_tkl) : 0;
    if (over_budget(ctx, tkl_bytes(cap) - old)) {
        cap = n;
        if (over_budget(ctx, tkl_bytes(cap) - old)) return TRD_EBUDGET;
    }
    free_tkl(ctx);
    ctx->bytes -= old;
    ctx->cap_tkl = 0;
    int64_t acc = 0;
    int rc;
    const int64_t hl = tkl_hist_len(cap);
    if ((rc = dev_alloc(ctx, &ctx->d_keys_a, cap, &acc)) || (rc = dev_alloc(ctx, &ctx->d_keys_b, cap, &acc)) ||
        (rc = dev_alloc(ctx, &ctx->d_sorted, cap, &acc)) || (rc = dev_alloc(ctx, &ctx->d_tmp, cap, &acc)) ||
        (rc = dev_alloc(ctx, &ctx->d_hist, hl, &acc)) || (rc = dev_alloc(ctx, &ctx->d_hist_off, hl, &acc)) ||
        (rc = dev_alloc(ctx, &ctx->d_tiles_tkl, scan_block_sums_len(hl), &acc))) {
        free_tkl(ctx);
        return rc;
    }
    ctx->bytes += tkl_bytes(cap);
    ctx->cap_tkl = cap;
    return TRD_OK;
}

int ensure_cells(trd_ctx *ctx, int64_t nc)
{
    if (nc <= ctx->cap_cells && ctx->d_offsets) return TRD_OK;
    const int64_t old = ctx->d_offsets ? cell_bytes(ctx->cfg, ctx->cap_cells) : 0;
    if (over_budget(ctx, cell_bytes(ctx->cfg, nc) - old)) return TRD_EBUDGET;
    dev_free(&ctx->d_offsets);
    ctx->bytes -= old;
    ctx->cap_cells = 0;
    int64_t acc = 0;
    const int rc = dev_alloc(ctx, &ctx->d_offsets, cell_entries(ctx->cfg, nc), &acc);
    if (rc) return rc;
    ctx->bytes += cell_bytes(ctx->cfg, nc);
    ctx->cap_cells = nc;
    return TRD_OK;
}

void free_trk(trd_ctx *ctx)
{
    dev_free(&ctx->d_fb);
    dev_free(&ctx->d_tkey_a);
    dev_free(&ctx->d_tkey_b);
    dev_free(&ctx->d_tval_a);
    dev_free(&ctx->d_tval_b);
    dev_free(&ctx->d_trank);
    dev_free(&ctx->d_thist);
    dev_free(&ctx->d_thist_off);
    dev_free(&ctx->d_ttiles);
    dev_free(&ctx->d_rows_in);
    dev_free(&ctx->d_rows_out);
}

int ensure_trk(trd_ctx *ctx, int64_t n)
{
    if (n <= ctx->cap_trk && ctx->d_fb) return TRD_OK;
    const trd_config &c = ctx->cfg;
    int64_t cap = n > 2 * ctx->cap_trk ? n : 2 * ctx->cap_trk;
    const int64_t old = ctx->d_fb ? trk_bytes(c, ctx->cap_trk) : 0;
    if (over_budget(ctx, trk_bytes(c, cap) - old)) {
        cap = n;
        if (over_budget(ctx, trk_bytes(c, cap) - old)) return TRD_EBUDGET;
    }
    free_trk(ctx);
    ctx->bytes -= old;
    ctx->cap_trk = 0;
    int64_t acc = 0;
    int rc = dev_alloc(ctx, &ctx->d_fb, cap, &acc);
    if (!rc && ordered(c)) {
        const int64_t hl = hist_len(cap), rs = row_scalar(c);
        (void)((rc = dev_alloc(ctx, &ctx->d_tkey_a, cap, &acc)) || (rc = dev_alloc(ctx, &ctx->d_tkey_b, cap, &acc)) ||
               (rc = dev_alloc(ctx, &ctx->d_tval_a, cap, &acc)) || (rc = dev_alloc(ctx, &ctx->d_tval_b, cap, &acc)) ||
               (rc = dev_alloc(ctx, &ctx->d_trank, cap, &acc)) || (rc = dev_alloc(ctx, &ctx->d_thist, hl, &acc)) ||
               (rc = dev_alloc(ctx, &ctx->d_thist_off, hl, &acc)) ||
               (rc = dev_alloc(ctx, &ctx->d_ttiles, scan_block_sums_len(hl), &acc)) ||
               (rc = dev_alloc(ctx, &ctx->d_rows_in, cap * kRowIn * rs, &acc)) ||
               (rc = dev_alloc(ctx, &ctx->d_rows_out, cap * kRowOut * rs, &acc)));
    }
    if (rc) {
        free_trk(ctx);
        return rc;
    }
    ctx->bytes += trk_bytes(c, cap);
    ctx->cap_trk = cap;
    return TRD_OK;
}

int64_t n_cells_of(const trd_config &c, int32_t ng)
{
    return (int64_t)ng * TRD_N_DET * c.n_rows * c.n_db * c.n_yb;
}

int launch_status()
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TRD_OK : TRD_EDEVICE;
}

// Errors left by earlier work, reported before anything is enqueued: the
// calling thread's pending HIP error (a failed launch or call), then an
// error that work already on the stream ran into (a fault in an enqueued
// kernel surfaces there once the stream reaches it).  A stream being
// captured into a graph is not queried (that would end the capture).
// Either error is consumed and reported as TRD_EDEVICE.
int pending_status(hipStream_t s)
{
    if (hipPeekAtLastError() != hipSuccess) {
        (void)hipGetLastError();
        return TRD_EDEVICE;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return TRD_EDEVICE;
    }
    if (cs == hipStreamCaptureStatusNone) {
        const hipError_t e = hipStreamQuery(s);
        // the query may record "not ready" as the thread's last error: clear
        // it either way so that the launch check after this call sees only
        // its own launches
        (void)hipGetLastError();
        if (e != hipSuccess && e != hipErrorNotReady) return TRD_EDEVICE;
    }
    return TRD_OK;
}

}  // namespace

extern "C" {

int trd_create(const trd_config *cfg, int device, trd_ctx **out)
{
    if (!out) return TRD_EINVAL;
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    if (cfg->flags & TRD_CFG_FAIL_ALLOC) return TRD_ENOMEM;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return device < 0 ? TRD_EINVAL : TRD_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return TRD_EDEVICE;
    if ((rc = scratch_setup(device))) return rc;
    trd_ctx *ctx = new (std::nothrow) trd_ctx();
    if (!ctx) return TRD_ENOMEM;
    ctx->device = device;
    ctx->cfg = *cfg;
    int64_t acc = 0;
    if ((rc = dev_alloc(ctx, &ctx->d_dx64, TRD_N_DET, &acc)) ||
        (rc = dev_alloc(ctx, &ctx->d_dx32, TRD_N_DET, &acc)) ||
        (rc = dev_alloc(ctx, &ctx->d_small, 4, &acc))) {
        trd_destroy(ctx);
        return rc;
    }
    ctx->bytes += acc;
    float dx32[TRD_N_DET];
    for (int d = 0; d < TRD_N_DET; d++) dx32[d] = (float)cfg->dx_chamber[d];
    if (hipMemcpy(ctx->d_dx64, cfg->dx_chamber, sizeof(double) * TRD_N_DET, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(ctx->d_dx32, dx32, sizeof(float) * TRD_N_DET, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(ctx->d_small, 0, 4 * sizeof(uint32_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        trd_destroy(ctx);
        return TRD_EDEVICE;
    }
    if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        ctx->n_cu = 1;
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming) != hipSuccess) {
        trd_destroy(ctx);
        return TRD_EDEVICE;
    }
    if (cfg->flags & TRD_CFG_TIME_KERNEL) {
        for (int k = 0; k < trd_ctx::kEvRing; k++)
            if (hipEventCreate(&ctx->ev[k][0]) != hipSuccess || hipEventCreate(&ctx->ev[k][1]) != hipSuccess) {
                trd_destroy(ctx);
                return TRD_EDEVICE;
            }
    }
    fill_devcfg(ctx->gd, *cfg, (const double *)ctx->d_dx64);
    fill_devcfg(ctx->gf, *cfg, (const float *)ctx->d_dx32);
    if (ctx->cfg.block_size == 0) ctx->cfg.block_size = 256;
    if (ctx->cfg.search_lanes == 0) ctx->cfg.search_lanes = 1;
    *out = ctx;
    return TRD_OK;
}

int trd_reserve(trd_ctx *ctx, int64_t max_tracklets, int32_t max_groups, int64_t max_tracks)
{
    if (!ctx || max_tracklets < 0 || max_groups < 1 || max_tracks < 0) return TRD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    const int64_t nc = n_cells_of(ctx->cfg, max_groups);
    if (nc >= (int64_t)UINT32_MAX - 1 || max_tracklets >= (int64_t)INT32_MAX) return TRD_EINVAL;
    int rc;
    if ((rc = ensure_tkl(ctx, max_tracklets)) || (rc = ensure_cells(ctx, nc)) ||
        (rc = ensure_trk(ctx, max_tracks)))
        return rc;
    return hip_status(hipDeviceSynchronize());
}

}  // extern "C"

namespace {

int load_check(const trd_ctx *ctx, const trd_tracklets *t, int64_t n, int32_t n_groups)
{
    if (!ctx || !t || n < 0 || n_groups < 1) return TRD_EINVAL;
    if (n > 0 && (!t->y || !t->z || !t->dy || !t->det_row)) return TRD_EINVAL;
    if (n >= (int64_t)INT32_MAX) return TRD_EINVAL;
    const int64_t nc = n_cells_of(ctx->cfg, n_groups);
    if (nc >= (int64_t)UINT32_MAX - 1) return TRD_EINVAL;
    return TRD_OK;
}

// Buffers of the binning, then its kernels on s (arguments checked).
int load_enqueue(trd_ctx *ctx, const trd_tracklets *t, int64_t n, int32_t n_groups, hipStream_t s)
{
    const int64_t nc = n_cells_of(ctx->cfg, n_groups);
    int rc;
    if ((rc = ensure_tkl(ctx, n)) || (rc = ensure_cells(ctx, nc))) return rc;
    BinCfg b = ctx->gd.bin;
    b.n_groups = n_groups;
    b.n_cells = (uint32_t)nc;
    ctx->gd.bin = b;
    ctx->gf.bin = b;
    BinBuffers buf{};
    buf.keys_a = ctx->d_keys_a;
    buf.keys_b = ctx->d_keys_b;
    buf.sorted = ctx->d_sorted;
    buf.recs_tmp = ctx->d_tmp;
    buf.hist = ctx->d_hist;
    buf.hist_off = ctx->d_hist_off;
    buf.tiles_tkl = ctx->d_tiles_tkl;
    buf.offsets = ctx->d_offsets;
    buf.bstart = ctx->d_offsets + ctx->cap_cells + 1;
    launch_bin(t->y, t->z, t->dy, t->det_row, t->group, n, b, buf, s);
    if ((rc = launch_status())) return rc;
    ctx->loaded = true;
    ctx->n_tkl = n;
    ctx->n_groups = n_groups;
    ctx->n_cells = nc;
    return TRD_OK;
}

}  // namespace

extern "C" {

int trd_load_tracklets(trd_ctx *ctx, const trd_tracklets *t, int64_t n, int32_t n_groups,
                       void *hip_stream)
{
    int rc;
    if ((rc = load_check(ctx, t, n, n_groups))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    hipStream_t s = (hipStream_t)hip_stream;
    if ((rc = pending_status(s))) return rc;
    return load_enqueue(ctx, t, n, n_groups, s);
}

}  // extern "C"

namespace {

// The launch sequence of trd_match.  With `fixed` (trd_match_noalloc) the
// re-run queue and the counters come from that scratch, the tracks are
// matched in the caller's order and nothing is allocated; otherwise the
// context's buffers are used (grown as needed).
int match_check(const trd_tracks *in, int64_t n, const trd_results *out)
{
    if (!in || !out || n < 0) return TRD_EINVAL;
    if (n == 0) return TRD_OK;
    if (n >= (int64_t)INT32_MAX) return TRD_EINVAL;
    if (!in->p || !in->cov || !in->x || !in->sector || !out->idx || !out->p || !out->cov ||
        !out->x || !out->sector || !out->chi2 || !out->n_match || !out->status)
        return TRD_EINVAL;
    return TRD_OK;
}

// A match call in parts: prepare (buffers, arguments of the kernels; `ord`:
// the call runs in the spatial order of the seeds of n_groups groups), the
// ordering of the seeds (sort and pack), and the match itself.
struct MatchCall {
    MatchIO io{};
    TrackOrder ob{};
    bool ord = false;
};

int match_prepare(trd_ctx *ctx, const trd_tracks *in, int64_t n, trd_results *out, int32_t n_groups,
                  uint32_t *fixed, MatchCall &mc)
{
    int rc;
    mc.ord = !fixed && ordered(ctx->cfg) && n_groups < kMaxOrderGroups;
    if (!fixed && (ctx->cfg.precision == TRD_PREC_FP32 || ordered(ctx->cfg)) && (rc = ensure_trk(ctx, n)))
        return rc;
    MatchIO &io = mc.io;
    io.sorted = ctx->d_sorted;
    io.offsets = ctx->d_offsets;
    io.ip = in->p;
    io.ic = in->cov;
    io.ix = in->x;
    io.isec = in->sector;
    io.igrp = in->group;
    io.n = n;
    io.oidx = out->idx;
    io.op = out->p;
    io.oc = out->cov;
    io.ox = out->x;
    io.osec = out->sector;
    io.ochi2 = out->chi2;
    io.ochi2l = out->chi2_layer;
    io.onm = out->n_match;
    io.ost = out->status;
    uint32_t *counters = fixed ? fixed : ctx->d_small;
    io.fb_list = fixed ? reinterpret_cast<int32_t *>(fixed + kScratchHead) : ctx->d_fb;
    io.fb_count = counters;
    io.fb_done = counters + 1;
    io.force_fallback = (ctx->cfg.flags & TRD_CFG_FORCE_FALLBACK) ? 1 : 0;
    io.work_next = counters + 2;
    io.work_done = counters + 3;
    if (mc.ord)
        mc.ob = TrackOrder{ctx->d_tkey_a, ctx->d_tkey_b, ctx->d_tval_a, ctx->d_tval_b, ctx->d_trank,
                           ctx->d_thist, ctx->d_thist_off, ctx->d_ttiles, ctx->d_rows_in, ctx->d_rows_out};
    return TRD_OK;
}

void match_order(trd_ctx *ctx, MatchCall &mc, int32_t n_groups, hipStream_t s)
{
    if (mc.ord) launch_order_in(ctx->cfg.precision, mc.io, n_groups, mc.ob, s);
}

int match_run(trd_ctx *ctx, MatchCall &mc, uint32_t *fixed, hipStream_t s)
{
    MatchIO &io = mc.io;
    // the shared scratch keeps the last call's contents: the counters start
    // at zero (a fill kernel, also under stream capture)
    if (fixed) launch_fill_u32(fixed, 0u, 4, s);
    if (ctx->cfg.flags & TRD_CFG_TIME_KERNEL) {
        const int slot = (int)(ctx->ev_count % trd_ctx::kEvRing);
        io.ev_begin = ctx->ev[slot][0];
        io.ev_end = ctx->ev[slot][1];
        ctx->ev_count++;
    }
    if (ctx->cfg.n_hyp > 0)
        launch_beam(ctx->cfg.precision, ctx->gd, ctx->gf, io, ctx->cfg.n_hyp, s);
    else
        launch_match(ctx->cfg.precision, ctx->gd, ctx->gf, io, ctx->cfg.block_size, ctx->cfg.search_lanes,
                     (ctx->cfg.flags & TRD_CFG_PERSISTENT) != 0, ctx->n_cu, s);
    if (mc.ord) launch_order_out(ctx->cfg.precision, io, mc.ob, s);
    return launch_status();
}

int match_impl(trd_ctx *ctx, const trd_tracks *in, int64_t n, trd_results *out, void *hip_stream,
               uint32_t *fixed)
{
    if (!ctx) return TRD_EINVAL;
    int rc;
    if ((rc = match_check(in, n, out))) return rc;
    if (!ctx->loaded) return TRD_ESTATE;
    if (n == 0) return TRD_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    const hipStream_t s = (hipStream_t)hip_stream;
    if ((rc = pending_status(s))) return rc;
    MatchCall mc;
    if ((rc = match_prepare(ctx, in, n, out, ctx->n_groups, fixed, mc))) return rc;
    match_order(ctx, mc, ctx->n_groups, s);
    return match_run(ctx, mc, fixed, s);
}

}  // namespace

extern "C" {

int trd_match(trd_ctx *ctx, const trd_tracks *in, int64_t n, trd_results *out, void *hip_stream)
{
    return match_impl(ctx, in, n, out, hip_stream, nullptr);
}

int trd_match_noalloc(trd_ctx *ctx, const trd_tracks *in, int64_t n, trd_results *out, void *hip_stream)
{
    if (!ctx) return TRD_EINVAL;
    if (n > kNoAllocMaxTracks) return TRD_EINVAL;
    uint32_t *sc = scratch_of(ctx->device);
    if (!sc) return ctx->device >= kMaxScratchDevices ? TRD_EINVAL : TRD_EDEVICE;
    return match_impl(ctx, in, n, out, hip_stream, sc);
}

int trd_load_and_match(trd_ctx *ctx, const trd_tracklets *t, int64_t n_tkl, int32_t n_groups,
                       const trd_tracks *in, int64_t n, trd_results *out, void *hip_stream)
{
    int rc;
    if ((rc = load_check(ctx, t, n_tkl, n_groups)) || (rc = match_check(in, n, out))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    const hipStream_t s = (hipStream_t)hip_stream;
    if ((rc = pending_status(s))) return rc;
    // every buffer first: the match reads the binning's at their final place
    if ((rc = ensure_tkl(ctx, n_tkl)) || (rc = ensure_cells(ctx, n_cells_of(ctx->cfg, n_groups)))) return rc;
    MatchCall mc;
    if (n > 0 && (rc = match_prepare(ctx, in, n, out, n_groups, nullptr, mc))) return rc;
    // the seeds' order on the side stream, from the point where the caller's
    // inputs are ready, beside the binning
    const bool fork = n > 0 && mc.ord;
    if (fork && (hipEventRecord(ctx->fork_ev, s) != hipSuccess ||
                 hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0) != hipSuccess))
        return TRD_EDEVICE;
    if (fork) match_order(ctx, mc, n_groups, ctx->side);
    if (fork && (hipEventRecord(ctx->join_ev, ctx->side) != hipSuccess || (rc = launch_status())))
        return rc ? rc : TRD_EDEVICE;
    // the stream joins the side stream before anything can fail, so that a
    // captured fork is always joined
    rc = load_enqueue(ctx, t, n_tkl, n_groups, s);
    if (fork && hipStreamWaitEvent(s, ctx->join_ev, 0) != hipSuccess) return TRD_EDEVICE;
    if (rc || n == 0) return rc;
    return match_run(ctx, mc, nullptr, s);
}

int trd_refit(trd_ctx *ctx, const trd_refit_in *in, const trd_tracklets *tkl, int64_t n_tkl, int64_t n,
              trd_refit_out *out, void *hip_stream)
{
    if (!ctx || !in || !tkl || !out || n < 0 || n_tkl < 0) return TRD_EINVAL;
    if (n == 0) return TRD_OK;
    if (n >= (int64_t)INT32_MAX || n_tkl >= (int64_t)INT32_MAX) return TRD_EINVAL;
    if (!in->p || !in->x || !in->sector || !in->idx || !out->p || !out->cov || !out->x || !out->sector ||
        !out->chi2 || !out->n_used || !out->status)
        return TRD_EINVAL;
    if (n_tkl > 0 && (!tkl->y || !tkl->z || !tkl->det_row)) return TRD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    if (int rc = pending_status((hipStream_t)hip_stream)) return rc;
    RefitIO io{};
    io.ip = in->p;
    io.ix = in->x;
    io.isec = in->sector;
    io.idx = in->idx;
    io.y = tkl->y;
    io.z = tkl->z;
    io.det_row = tkl->det_row;
    io.n = n;
    io.n_tkl = n_tkl;
    for (int k = 0; k < 5; k++) io.cov0[k] = ctx->cfg.refit_cov[k];
    io.min_tracklets = ctx->cfg.refit_min;
    io.op = out->p;
    io.oc = out->cov;
    io.ox = out->x;
    io.ochi2 = out->chi2;
    io.osec = out->sector;
    io.onused = out->n_used;
    io.ost = out->status;
    launch_refit(ctx->cfg.precision, ctx->gd, ctx->gf, io, (hipStream_t)hip_stream);
    return launch_status();
}

int trd_residual_sums(trd_ctx *ctx, const trd_reference *ref, const trd_tpc_clusters *cl, int64_t n,
                      int64_t n_cl, double *sums, void *hip_stream)
{
    if (!ctx || !ref || !cl || !sums || n < 0 || n_cl < 0) return TRD_EINVAL;
    if (n == 0) return TRD_OK;
    if (!ref->p || !ref->x || !ref->sector || !ref->status || !cl->first) return TRD_EINVAL;
    if (n_cl > 0 && (!cl->y || !cl->z || !cl->row_sec)) return TRD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    if (int rc = pending_status((hipStream_t)hip_stream)) return rc;
    const trd_config &c = ctx->cfg;
    ResidualIO io{};
    io.rp = ref->p;
    io.rx = ref->x;
    io.rsec = ref->sector;
    io.rstatus = ref->status;
    io.cy = cl->y;
    io.cz = cl->z;
    io.row_sec = cl->row_sec;
    io.first = cl->first;
    io.n = n;
    io.sums = sums;
    io.x_in = c.tpc_x_in;
    io.x_out = c.tpc_x_out;
    io.n_rows = c.tpc_n_rows;
    io.nx = c.vox_nx;
    io.ny = c.vox_ny;
    io.nz = c.vox_nz;
    io.nvox = TRD_N_SECTORS * c.vox_nx * c.vox_ny * c.vox_nz;
    launch_residual_sums(c.precision, ctx->gd, ctx->gf, io, ctx->n_cu, (hipStream_t)hip_stream);
    return launch_status();
}

int trd_voxel_solve(trd_ctx *ctx, const double *sums, float *dist, void *hip_stream)
{
    if (!ctx || !sums || !dist) return TRD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    if (int rc = pending_status((hipStream_t)hip_stream)) return rc;
    const trd_config &c = ctx->cfg;
    launch_voxel_solve(sums, TRD_N_SECTORS * c.vox_nx * c.vox_ny * c.vox_nz, c.vox_min, dist,
                       (hipStream_t)hip_stream);
    return launch_status();
}

int trd_get_binning(trd_ctx *ctx, trd_binning_view *out)
{
    if (!ctx || !out) return TRD_EINVAL;
    if (!ctx->loaded) return TRD_ESTATE;
    out->offsets = ctx->d_offsets;
    out->sorted = reinterpret_cast<const float *>(ctx->d_sorted);
    out->n_cells = ctx->n_cells;
    out->n_tracklets = ctx->n_tkl;
    return TRD_OK;
}

int trd_copy_binning(trd_ctx *ctx, uint32_t *offsets_out, float *sorted_out, int64_t max_valid,
                     void *hip_stream)
{
    if (!ctx || !offsets_out || (!sorted_out && max_valid > 0) || max_valid < 0) return TRD_EINVAL;
    if (!ctx->loaded) return TRD_ESTATE;
    if (max_valid < ctx->n_tkl) return TRD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    hipStream_t s = (hipStream_t)hip_stream;
    if (int rc = pending_status(s)) return rc;
    if (hipMemcpyAsync(offsets_out, ctx->d_offsets, sizeof(uint32_t) * (size_t)(ctx->n_cells + 1),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TRD_EDEVICE;
    if (ctx->n_tkl > 0 &&
        hipMemcpyAsync(sorted_out, ctx->d_sorted, sizeof(float4) * (size_t)ctx->n_tkl,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TRD_EDEVICE;
    return TRD_OK;
}

int64_t trd_device_bytes(const trd_ctx *ctx) { return ctx ? ctx->bytes : 0; }

int trd_kernel_times(trd_ctx *ctx, float *ms, int32_t max_n)
{
    if (!ctx || (max_n > 0 && !ms) || max_n < 0) return TRD_EINVAL;
    if (!(ctx->cfg.flags & TRD_CFG_TIME_KERNEL)) return TRD_ESTATE;
    if (hipSetDevice(ctx->device) != hipSuccess) return TRD_EDEVICE;
    int64_t have = ctx->ev_count < trd_ctx::kEvRing ? ctx->ev_count : trd_ctx::kEvRing;
    if (have > max_n) have = max_n;
    for (int64_t k = 0; k < have; k++) {
        const int slot = (int)((ctx->ev_count - have + k) % trd_ctx::kEvRing);
        if (hipEventSynchronize(ctx->ev[slot][1]) != hipSuccess ||
            hipEventElapsedTime(&ms[k], ctx->ev[slot][0], ctx->ev[slot][1]) != hipSuccess) {
            (void)hipGetLastError();
            return TRD_EDEVICE;
        }
    }
    ctx->ev_count = 0;
    return (int)have;
}

void trd_destroy(trd_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    dev_free(&ctx->d_dx64);
    dev_free(&ctx->d_dx32);
    dev_free(&ctx->d_small);
    free_tkl(ctx);
    dev_free(&ctx->d_offsets);
    free_trk(ctx);
    for (int k = 0; k < trd_ctx::kEvRing; k++)
        for (int e = 0; e < 2; e++)
            if (ctx->ev[k][e]) (void)hipEventDestroy(ctx->ev[k][e]);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    delete ctx;
}

const char *trd_status_string(int code)
{
    switch (code) {
    case TRD_OK: return "ok";
    case TRD_EINVAL: return "invalid argument";
    case TRD_ENOMEM: return "device allocation failed";
    case TRD_EDEVICE: return "HIP device error";
    case TRD_ESTATE: return "no tracklets loaded";
    case TRD_EBUDGET: return "HBM budget exceeded";
    default: return "unknown status";
    }
}

}  // extern "C"
