// noalloc.hip -- the projection forward for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation): the same kernels as
// digs_project_fwd, with the intermediate buffers in a fixed device array owned by the library
// instead of a caller workspace.
//
// The array is a file-scope __device__ variable: every GPU the library runs on holds its own copy,
// allocated when the code object loads and kept until the process ends. Its address on a device
// is looked up once per device with hipGetSymbolAddress (with that device current) and cached;
// host code uses only that address, never the variable's name. Calls on one GPU share the array,
// so calls that overlap on one GPU (different streams without ordering, or different threads)
// race; each call clears what must start at zero.
#include <mutex>

#include "kernels.h"
#include "prof.h"

static __device__ __align__(256) unsigned char scratch[DIGS_NOALLOC_SCRATCH_BYTES];

#define NOALLOC_MAX_DEVICES 64
static void *g_scratch[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mutex;

// The device address of this device's copy of `scratch` (looked up on the first call on it).
static int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return digs_set_hip_error(e);
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return DIGS_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return digs_set_hip_error(e != hipSuccess ? e : hipErrorUnknown);
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DIGS_OK;
}

__global__ void k_noalloc_diag_clear(DiagBlock *d) { diag_clear(d); }

// the public fields of the call's diagnostics, for the caller to read when it wants
__global__ void k_noalloc_diag_out(const DiagBlock *d, digs_diag *out)
{
    out->instances = d->instances;
    out->capacity = d->capacity;
    out->overflow = d->overflow;
    out->nonfinite = d->nonfinite;
    out->folded = d->folded;
    out->behind_source = d->behind_source;
    out->wide = d->wide;
    out->reserved0 = 0;
    out->max_instances = d->instances;
    for (int k = 0; k < 4; ++k) out->reserved[k] = 0;
}

extern "C" int digs_project_fwd_noalloc(const digs_geom *geom, const digs_grid *grid,
                                        const float *coef, int n, const float *mu,
                                        const float *scale, const float *quat, const float *rho,
                                        int T, const float *angles, const float *w, float *proj,
                                        digs_diag *diag_out, const digs_tuning *tuning,
                                        void *stream)
{
    // sizes first, on the host: a problem whose forward needs more than the array is rejected
    // before any device work
    WsLayout L;
    if (!ws_layout(geom, grid, n, T, tuning, &L, true)) return DIGS_EINVAL;
    if (L.total > (size_t)DIGS_NOALLOC_SCRATCH_BYTES) return DIGS_ESCRATCH;
    void *ptr = nullptr;
    int rc = scratch_address(&ptr);
    if (rc != DIGS_OK) return rc;
    RenderArgs a;
    rc = render_prepare(geom, grid, coef, n, mu, scale, quat, rho, T, angles, w, ptr,
                        (size_t)DIGS_NOALLOC_SCRATCH_BYTES, tuning, true, &a);
    if (rc != DIGS_OK) return rc;
    if (T > 0 && !proj) return DIGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    ProfSuppress no_events;   // no stage-timing events for this call
    DiagBlock *diag = reinterpret_cast<DiagBlock *>(a.ws + a.L.diag);
    hipLaunchKernelGGL(k_noalloc_diag_clear, dim3(1), dim3(1), 0, s, diag);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && T > 0) {
        if (n == 0) {
            e = render_zero(proj, (size_t)T * geom->nu * geom->nv, s);
        } else {
            e = render_forward_setup(a, s);
            if (e == hipSuccess) e = render_forward_splat(a, proj, s);
        }
    }
    if (e == hipSuccess && diag_out) {
        hipLaunchKernelGGL(k_noalloc_diag_out, dim3(1), dim3(1), 0, s, diag, diag_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? DIGS_OK : digs_set_hip_error(e);
}
