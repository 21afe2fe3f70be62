// C-ABI entry points (include/clusco.h): argument validation, workspace
// layout and the launch sequence.  Every argument error is caught here,
// before anything is enqueued; nothing here allocates device memory or
// synchronises the host (clusco_fixup_count excepted).
#include <string.h>

#include <string>

#include "internal.h"

using namespace clusco;

struct clusco_ctx {
    int device;
    double tol[4];   // fix-up tolerance per precision (A); <= 0 disables
    double eps[4];   // calibrated relative error of the contraction per precision
    std::string last_error;
};

namespace {

constexpr int64_t MAX_N = 1 << 20;   // packed list entries hold 16-bit row blocks

clusco_status fail(clusco_handle h, clusco_status s, const char *msg)
{
    if (h) h->last_error = msg;
    return s;
}

clusco_status hip_fail(clusco_handle h, hipError_t e, const char *where)
{
    if (h) {
        h->last_error = where;
        h->last_error += ": ";
        h->last_error += hipGetErrorString(e);
    }
    return CLUSCO_ERR_HIP;
}

bool valid_precision(clusco_precision p)
{
    return p == CLUSCO_FP32 || p == CLUSCO_SPLIT_BF16 || p == CLUSCO_SPLIT_FP16 || p == CLUSCO_FP64;
}

int mode_of(clusco_precision p)
{
    switch (p) {
    case CLUSCO_FP32: return MODE_FP32;
    case CLUSCO_SPLIT_BF16: return MODE_BF16;
    case CLUSCO_SPLIT_FP16: return MODE_FP16;
    default: return MODE_FP64;
    }
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

double flag_coef(clusco_handle h, int mode, int64_t L)
{
    const double tol = h->tol[mode];
    if (!(tol > 0.0)) return -1.0;
    // flag when  eps (E_i + E_j) / (L score) > tol / 2
    return 2.0 * h->eps[mode] / ((double)L * tol);
}

} // namespace

extern "C" {

const char *clusco_status_string(clusco_status s)
{
    switch (s) {
    case CLUSCO_OK: return "CLUSCO_OK";
    case CLUSCO_ERR_INVALID_ARG: return "CLUSCO_ERR_INVALID_ARG";
    case CLUSCO_ERR_WORKSPACE: return "CLUSCO_ERR_WORKSPACE";
    case CLUSCO_ERR_UNSUPPORTED: return "CLUSCO_ERR_UNSUPPORTED";
    case CLUSCO_ERR_HIP: return "CLUSCO_ERR_HIP";
    }
    return "CLUSCO_ERR_UNKNOWN";
}

clusco_status clusco_create(clusco_handle *h, int device)
{
    if (!h || device < 0) return CLUSCO_ERR_INVALID_ARG;
    clusco_ctx *c = new (std::nothrow) clusco_ctx;
    if (!c) return CLUSCO_ERR_INVALID_ARG;
    c->device = device;
    c->tol[MODE_FP32] = 1e-4;
    c->tol[MODE_BF16] = 5e-4;
    c->tol[MODE_FP16] = 1e-4;
    c->tol[MODE_FP64] = 1e-6;
    c->eps[MODE_FP32] = 3e-7;
    c->eps[MODE_BF16] = 7e-7;
    c->eps[MODE_FP16] = 1.6e-7;
    c->eps[MODE_FP64] = 0.0;
    *h = c;
    return CLUSCO_OK;
}

void clusco_destroy(clusco_handle h) { delete h; }

const char *clusco_last_error(clusco_handle h) { return h ? h->last_error.c_str() : ""; }

clusco_status clusco_set_tolerance(clusco_handle h, clusco_precision p, double tol)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    h->tol[mode_of(p)] = tol;
    return CLUSCO_OK;
}

size_t clusco_crmsd_workspace_size(clusco_handle h, int64_t N, int64_t L, clusco_precision p)
{
    if (!h || N < 0 || N > MAX_N || L < 1 || !valid_precision(p)) return 0;
    return fwd_layout(mode_of(p), N, L).total;
}

clusco_status clusco_crmsd_matrix(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                  clusco_precision p, float *out, void *ws, size_t ws_bytes,
                                  void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (N < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0 and L >= 1");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (N < 2) return CLUSCO_OK;
    if (!coords || !out) return fail(h, CLUSCO_ERR_INVALID_ARG, "null coords or out");
    if (!aligned(coords, 4) || !aligned(out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "coords and out must be 4-byte aligned");
    const int mode = mode_of(p);
    const FwdLayout f = fwd_layout(mode, N, L);
    if (!ws || ws_bytes < f.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");

    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int *counter = (int *)(w + f.off_counter);
    double *E = (double *)(w + f.off_E);
    double *cen = (double *)(w + f.off_cen);

    PrepArgs pa{coords, N, L, f.Np, f.Lp, f.KB, w + f.off_ops, E, cen, counter};
    hipError_t e = launch_prep(mode, pa, s);
    if (e != hipSuccess) return hip_fail(h, e, "prep launch");

    const double coef = flag_coef(h, mode, L);
    if (mode != MODE_FP64) {
        TileArgs ta{};
        ta.ops = w + f.off_ops;
        ta.E = E;
        ta.N = N;
        ta.L = L;
        ta.Np = f.Np;
        ta.KB = f.KB;
        ta.nb = f.Np / TILE;
        ta.T = tri_count(ta.nb);
        ta.out = out;
        ta.flag_coef = coef;
        ta.counter = counter;
        ta.list = (uint32_t *)(w + f.off_list);
        e = launch_tile(mode, ta, s);
        if (e != hipSuccess) return hip_fail(h, e, "tile launch");
        if (coef > 0.0) {
            FixupArgs fa{coords, cen, E, N, L, f.nrb, out, coef, counter,
                         (const uint32_t *)(w + f.off_list), 0};
            e = launch_fixup(fa, s);
            if (e != hipSuccess) return hip_fail(h, e, "fixup launch");
        }
    } else {
        FixupArgs fa{coords, cen, E, N, L, f.nrb, out, 0.0, nullptr, nullptr, f.n_wave_tiles};
        e = launch_fixup(fa, s);
        if (e != hipSuccess) return hip_fail(h, e, "fp64 launch");
    }
    return CLUSCO_OK;
}

clusco_status clusco_fixup_count(clusco_handle h, const void *ws, int64_t *count, void *stream)
{
    if (!h || !ws || !count) return CLUSCO_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    int v = 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&v, ws, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "read fix-up counter");
    *count = v;
    return CLUSCO_OK;
}

} // extern "C"
