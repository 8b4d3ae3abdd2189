// api.cpp -- contexts, status strings, one-shot solves and diagnostics.
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace lbmh;

extern "C" lbm_status lbm_solver_create_ex(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls,
                                           const lbm_params *pp, int require_percolation,
                                           lbm_solver **out);

extern "C" {

const char *lbm_status_str(int status)
{
    switch (status) {
    case LBM_OK:
        return "LBM_OK";
    case LBM_NOT_CONVERGED:
        return "LBM_NOT_CONVERGED";
    case LBM_STALLED:
        return "LBM_STALLED";
    case LBM_EINVAL:
        return "LBM_EINVAL";
    case LBM_ENOMEM:
        return "LBM_ENOMEM";
    case LBM_EDEVICE:
        return "LBM_EDEVICE";
    case LBM_EDIVERGED:
        return "LBM_EDIVERGED";
    case LBM_EBUSY:
        return "LBM_EBUSY";
    case LBM_ENOTFOUND:
        return "LBM_ENOTFOUND";
    default:
        return "LBM_UNKNOWN";
    }
}

const char *lbm_version(void)
{
    return "mfc-lbm-mi355x 0.1 (gfx950)";
}

lbm_status lbm_ctx_create(int device, void *hip_stream, lbm_ctx **out)
{
    if (!out)
        return LBM_EINVAL;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0)
        return LBM_EDEVICE;
    if (device < 0 || device >= count)
        return LBM_EINVAL;
    if ((e = hipSetDevice(device)) != hipSuccess)
        return LBM_EDEVICE;
    lbm_ctx *c = new lbm_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
            delete c;
            return LBM_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return LBM_OK;
}

void lbm_ctx_destroy(lbm_ctx *ctx)
{
    if (!ctx)
        return;
    if (ctx->own_stream && ctx->stream) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
}

const char *lbm_last_error(const lbm_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "";
}

void *lbm_ctx_stream(lbm_ctx *ctx)
{
    return ctx ? static_cast<void *>(ctx->stream) : nullptr;
}

lbm_status lbm_fluid_steady(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, double tau, double u_in,
                            double tol, int64_t max_iter, int storage, double *u_out, lbm_info *info)
{
    if (!ctx || !cls || !u_out)
        return set_err(ctx, LBM_EINVAL, "null argument");
    lbm_params p;
    memset(&p, 0, sizeof(p));
    p.tau = tau;
    p.u_in = u_in;
    p.D = 1.0 / 6.0; // unused by a fluid solve
    p.c_in = 1.0;
    p.storage = storage;
    p.check_every = 0; // the library default for the storage
    lbm_solver *s = nullptr;
    lbm_status st = lbm_solver_create(ctx, g, cls, &p, &s);
    if (st)
        return st;
    lbm_status r = lbm_solver_fluid(s, tol, max_iter, 0, info);
    if (r >= 0) {
        lbm_status e = lbm_solver_get(s, LBM_FIELD_U, u_out);
        if (e)
            r = e;
    }
    lbm_solver_destroy(s);
    return r;
}

lbm_status lbm_ad_steady(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const double *u, double D,
                         double c_in, double k_sink, int outlet, double c_out, double tol,
                         int64_t max_iter, int storage, double *c_field, lbm_info *info)
{
    if (!ctx || !cls || !u || !c_field)
        return set_err(ctx, LBM_EINVAL, "null argument");
    lbm_params p;
    memset(&p, 0, sizeof(p));
    p.tau = 1.0;   // unused by a substrate solve
    p.u_in = 0.01; // unused by a substrate solve
    p.D = D;
    p.c_in = c_in;
    p.k_sink = k_sink;
    p.outlet = outlet;
    p.c_out = c_out;
    p.storage = storage;
    p.check_every = 0; // the library default for the storage
    lbm_solver *s = nullptr;
    lbm_status st = lbm_solver_create_ex(ctx, g, cls, &p, 0, &s);
    if (st)
        return st;
    lbm_status r = lbm_solver_set_u(s, u);
    if (r == LBM_OK)
        r = lbm_solver_ad(s, tol, max_iter, 0, info);
    if (r >= 0) {
        lbm_status e = lbm_solver_get(s, LBM_FIELD_C, c_field);
        if (e)
            r = e;
    }
    lbm_solver_destroy(s);
    return r;
}

// the mask of a device-pointer call, staged to the host (geometry is host work)
static lbm_status mask_from_device(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, std::vector<uint8_t> &out)
{
    if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0)
        return set_err(ctx, LBM_EINVAL, "bad grid");
    out.resize((size_t)g.nx * g.ny * g.nz);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = stream_copy(ctx, out.data(), cls, out.size(), hipMemcpyDeviceToHost);
    return e == hipSuccess ? LBM_OK : hip_err(ctx, e, "mask copy");
}

lbm_status lbm_fluid_steady_dev(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, double tau,
                                double u_in, double tol, int64_t max_iter, int storage,
                                double *u_out, lbm_info *info)
{
    if (!ctx || !cls || !u_out)
        return set_err(ctx, LBM_EINVAL, "null argument");
    std::vector<uint8_t> mask;
    lbm_status st = mask_from_device(ctx, g, cls, mask);
    if (st)
        return st;
    lbm_params p;
    memset(&p, 0, sizeof(p));
    p.tau = tau;
    p.u_in = u_in;
    p.D = 1.0 / 6.0; // unused by a fluid solve
    p.c_in = 1.0;
    p.storage = storage;
    p.check_every = 0; // the library default for the storage
    lbm_solver *s = nullptr;
    if ((st = lbm_solver_create(ctx, g, mask.data(), &p, &s)))
        return st;
    lbm_status r = lbm_solver_fluid(s, tol, max_iter, 0, info);
    if (r >= 0) {
        lbm_status e = get_field_device(s, LBM_FIELD_U, u_out);
        if (e)
            r = e;
    }
    lbm_solver_destroy(s);
    return r;
}

lbm_status lbm_ad_steady_dev(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const double *u,
                             double D, double c_in, double k_sink, int outlet, double c_out,
                             double tol, int64_t max_iter, int storage, double *c_field,
                             lbm_info *info)
{
    if (!ctx || !cls || !u || !c_field)
        return set_err(ctx, LBM_EINVAL, "null argument");
    std::vector<uint8_t> mask;
    lbm_status st = mask_from_device(ctx, g, cls, mask);
    if (st)
        return st;
    lbm_params p;
    memset(&p, 0, sizeof(p));
    p.tau = 1.0;   // unused by a substrate solve
    p.u_in = 0.01; // unused by a substrate solve
    p.D = D;
    p.c_in = c_in;
    p.k_sink = k_sink;
    p.outlet = outlet;
    p.c_out = c_out;
    p.storage = storage;
    p.check_every = 0; // the library default for the storage
    lbm_solver *s = nullptr;
    if ((st = lbm_solver_create_ex(ctx, g, mask.data(), &p, 0, &s)))
        return st;
    lbm_status r = set_u_device(s, u);
    if (r == LBM_OK)
        r = lbm_solver_ad(s, tol, max_iter, 0, info);
    if (r >= 0) {
        lbm_status e = get_field_device(s, LBM_FIELD_C, c_field);
        if (e)
            r = e;
    }
    lbm_solver_destroy(s);
    return r;
}

lbm_status lbm_copy_bandwidth(lbm_ctx *ctx, size_t bytes, int reps, double *gbps, double *ms_per_copy)
{
    if (!ctx || bytes < 16 || reps < 1)
        return set_err(ctx, LBM_EINVAL, "bytes >= 16 and reps >= 1 required");
    bytes &= ~(size_t)15;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return hip_err(ctx, e, "set device");
    void *a = nullptr, *b = nullptr;
    if ((e = hipMalloc(&a, bytes)) != hipSuccess)
        return hip_err(ctx, e, "copy buffer");
    if ((e = hipMalloc(&b, bytes)) != hipSuccess) {
        (void)hipFree(a);
        return hip_err(ctx, e, "copy buffer");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lbm_status st = LBM_OK;
    float ms = 0.f;
    if ((e = hipMemsetAsync(a, 1, bytes, ctx->stream)) != hipSuccess ||
        (e = lbmk::copy_kernel(a, b, bytes, ctx->stream)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
        (e = hipEventRecord(e0, ctx->stream)) != hipSuccess) {
        st = hip_err(ctx, e, "copy setup");
    } else {
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = lbmk::copy_kernel((r & 1) ? b : a, (r & 1) ? a : b, bytes, ctx->stream);
        if (e == hipSuccess)
            e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess)
            st = hip_err(ctx, e, "copy timing");
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (st == LBM_OK) {
        const double per = ms / reps;
        if (ms_per_copy)
            *ms_per_copy = per;
        if (gbps)
            *gbps = 2.0 * (double)bytes / (per * 1e-3) / 1e9;
    }
    return st;
}

} // extern "C"
