// nh_solve_noalloc: the plain solve for callers that cannot allocate memory.
//
// Its device buffers - the counter and statistics words, the fused
// quadrature's sums and the staged inputs of one request - live in `scratch`,
// a file-scope device array of NOALLOC_SCRATCH_BYTES that each GPU the library
// runs on holds until the process ends; the inputs are staged on the host in a
// static array of the same size.  The kernels are those of nh_solve_async
// without a ratio buffer (the fused quadrature), so the profile is the same
// bits.  Every call on a GPU shares that GPU's scratch: calls that overlap on
// one GPU race (the host staging is serialised; the device work is not).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "nh_context.h"
#include "nh_launch.h"

namespace nh {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)4 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static unsigned char h_stage_static[NOALLOC_SCRATCH_BYTES];
static std::mutex g_noalloc_mu;
static void *g_scratch_dev[NOALLOC_MAX_DEVICES];   // scratch's address on each device

// The device address of `scratch` on the current device, looked up once per
// device (host code must not pass the array's name itself: on the host it is
// only a stand-in for the symbol).  Called under g_noalloc_mu.
static int scratch_on(nh_context *ctx, unsigned char **dev)
{
    if (ctx->device < 0 || ctx->device >= NOALLOC_MAX_DEVICES)
        return set_err(ctx, NH_EINVAL, "device %d beyond the %d the allocation-free entry point serves", ctx->device,
                       NOALLOC_MAX_DEVICES);
    if (!g_scratch_dev[ctx->device]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_dev[ctx->device] = p;
    }
    *dev = (unsigned char *)g_scratch_dev[ctx->device];
    return NH_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace nh

using namespace nh;

extern "C" size_t nh_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" int nh_solve_noalloc(nh_context *ctx, const nh_request *req, double *d_out, void *stream)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (!d_out || !req) return set_err(ctx, NH_EINVAL, "req and d_out are required");
    // before validation, whose check of sampled histories allocates
    if (req->halo.mass_kind == NH_MASS_TABLE || req->halo.conc_kind == NH_CONC_TABLE ||
        req->halo.kappa_kind == NH_KAPPA_TABLE)
        return set_err(ctx, NH_EINVAL, "sampled histories need the host spline set-up of nh_solve_async");
    int rc = validate(req, ctx->err, sizeof(ctx->err));
    if (rc != NH_OK) return rc;
    const Staged s = stage_layout(req, ctx->table_nodes, 0);
    // scratch layout: counter and statistics words, the quadrature sums, the staged inputs
    const size_t off_quad = 256;
    const size_t off_blob = align256(off_quad + quad_bytes(req->grid.n_r));
    const size_t total = off_blob + s.bytes;
    if (total > NOALLOC_SCRATCH_BYTES)
        return set_err(ctx, NH_EINVAL, "the request needs %zu bytes of scratch; the allocation-free entry point has %zu",
                       total, NOALLOC_SCRATCH_BYTES);

    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if ((rc = wait_pending(ctx)) != NH_OK) return rc;
    ctx->pending = false;
    unsigned char *dev = nullptr;
    if ((rc = scratch_on(ctx, &dev)) != NH_OK) return rc;

    TrajParams P;
    stage_fill(req, s, (char *)h_stage_static, P, 1);
    if (!ctx->free_exit && P.r_exit > 0.0) {
        P.r_exit = -1.0;
        P.cull_D = 0.0;
    }
    // a pageable source: the copy has read it when the call returns
    HIPCHK(hipMemcpyAsync(dev + off_blob, h_stage_static, s.bytes, hipMemcpyHostToDevice, st));
    SolveBufs b{};
    b.blob = (char *)(dev + off_blob);
    b.small = (unsigned long long *)dev;
    b.qa = quad_acc(dev + off_quad, req->grid.n_r, b.small + 8);
    return solve_launch(ctx, req, s, P, b, d_out, st, 0, nullptr);
}
