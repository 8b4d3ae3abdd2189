// noalloc.hip -- the steady fluid solve without device allocation.
//
// lbm_fluid_steady_dev_noalloc is lbm_fluid_steady_dev for callers that
// cannot allocate device memory (code under stream capture elsewhere in the
// program, tight serving loops, harnesses that forbid allocation).  Every
// device buffer of the solve -- the node descriptors, both population
// buffers, the velocity and its check history, the control block, the
// per-block check maxima, the column references and the flux partials -- is
// carved from `scratch`, a file-scope device array of LBM_NOALLOC_SCRATCH_BYTES
// that each GPU holds from the library's first use on it until the process
// ends.  The solve runs the same kernels in the same launch order as the
// allocating form, so its results are the same bit for bit; it reads each
// chunk's control block after a stream synchronisation instead of through
// events and pinned memory.
//
// Calls on one GPU share that GPU's array: calls that overlap on one GPU
// (from several threads or streams) race and must be serialised by the
// caller.  Each call clears the buffers it uses before the solve.
#include <string.h>

#include <mutex>
#include <vector>

#include "lbm_internal.h"

using namespace lbmh;

namespace {

static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

// Device address of this GPU's scratch array: looked up once per device
// with that device current (the array's name is a host-side stand-in, not
// a device address).
lbm_status scratch_of(lbm_ctx *ctx, void **out)
{
    if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
        return set_err(ctx, LBM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[ctx->device]) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return hip_err(ctx, e, "set device");
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_err(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        scratch_ptr[ctx->device] = p;
    }
    *out = scratch_ptr[ctx->device];
    return LBM_OK;
}

} // namespace

extern "C" {

lbm_status lbm_fluid_steady_dev_noalloc(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, double tau,
                                        double u_in, double tol, int64_t max_iter, int storage,
                                        double *u_out, lbm_info *info)
{
    if (!ctx || !cls || !u_out)
        return set_err(ctx, LBM_EINVAL, "null argument");
    if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0)
        return set_err(ctx, LBM_EINVAL, "bad grid");
    void *arena = nullptr;
    lbm_status st = scratch_of(ctx, &arena);
    if (st)
        return st;
    // the mask is read back once (geometry and link words are built on the
    // host), as in the allocating form
    std::vector<uint8_t> mask((size_t)g.nx * g.ny * g.nz);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = stream_copy(ctx, mask.data(), cls, mask.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_err(ctx, e, "mask copy");
    lbm_params p;
    memset(&p, 0, sizeof(p));
    p.tau = tau;
    p.u_in = u_in;
    p.D = 1.0 / 6.0; // unused by a fluid solve
    p.c_in = 1.0;
    p.storage = storage;
    p.check_every = 0; // the library default for the storage
    lbm_solver *s = nullptr;
    if ((st = solver_create_in(ctx, g, mask.data(), p, arena, LBM_NOALLOC_SCRATCH_BYTES, &s)))
        return st;
    lbm_status r = lbm_solver_fluid(s, tol, max_iter, 0, info);
    if (r >= 0) {
        lbm_status x = export_u_device(s, u_out);
        if (x)
            r = x;
    }
    lbm_solver_destroy(s); // synchronises the stream; frees nothing
    return r;
}

} // extern "C"
