// Allocation-free forward solve of a uniform batch (every problem n x p),
// for callers that cannot allocate device memory.  The work queue's
// counter and the per-problem metadata that a plan keeps in memory it
// allocates live here in one fixed device array, `scratch`, filled by a
// kernel on the caller's stream before each solve; the solve runs the
// wavefront kernel with X resident in LDS (no HBM workspace).
#include "ladl_host.hpp"
#include "ladl_kernels.hpp"
#include "ladlasso.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

namespace {

constexpr size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t MAXP = LADL_NOALLOC_MAX_PROBLEMS;
// byte offsets of the sections of `scratch`
constexpr size_t OFF_COUNTER = 0;                               // int32 queue head
constexpr size_t OFF_ROW = 256;                                 // int64 [MAXP + 1] row_off
constexpr size_t OFF_XOFF = OFF_ROW + al256(8 * (MAXP + 1));    // int64 [MAXP] x_off
constexpr size_t OFF_BOFF = OFF_XOFF + al256(8 * MAXP);         // int64 [MAXP] b_off
constexpr size_t OFF_P = OFF_BOFF + al256(8 * MAXP);            // int32 [MAXP] p
constexpr size_t OFF_ORDER = OFF_P + al256(4 * MAXP);           // int32 [MAXP] queue order
constexpr size_t SCRATCH_BYTES = OFF_ORDER + al256(4 * MAXP);   // 2.1 MB

constexpr int MAX_DEVICES = 64;

} // namespace

// One copy per GPU, held until the process ends.  Host code never uses
// this name as an address: it reads the device address of each GPU's copy
// with hipGetSymbolAddress once per device and passes that to kernels.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

__global__ void k_noalloc_setup(unsigned char *base, int P, int n, int p)
{
    int32_t *counter = (int32_t *)(base + OFF_COUNTER);
    int64_t *row_off = (int64_t *)(base + OFF_ROW);
    int64_t *x_off = (int64_t *)(base + OFF_XOFF);
    int64_t *b_off = (int64_t *)(base + OFF_BOFF);
    int32_t *p_arr = (int32_t *)(base + OFF_P);
    int32_t *order = (int32_t *)(base + OFF_ORDER);
    const int stride = gridDim.x * blockDim.x;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= P; k += stride) {
        row_off[k] = (int64_t)k * n;
        if (k < P) {
            x_off[k] = (int64_t)k * n * p;
            b_off[k] = (int64_t)k * p;
            p_arr[k] = p;
            order[k] = k; // equal cost: queue in problem order
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

struct DeviceScratch {
    unsigned char *ptr = nullptr; // device address of this GPU's `scratch`
    int num_cu = 0;
    size_t lds_max = 0;
};

std::mutex g_mu;
DeviceScratch g_dev[MAX_DEVICES];

int rows_per_lane(int n)
{
    int r = (n + 63) / 64, R = 1;
    while (R < r) R <<= 1;
    return R;
}

// the scratch address and launch limits of the current device, looked up
// once per device with that device current
int device_scratch(DeviceScratch &out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ladl::host_hipfail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return ladl::host_fail(LADL_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceScratch &d = g_dev[dev];
    if (!d.ptr) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return ladl::host_hipfail(e, "hipGetSymbolAddress(scratch)");
        int cu = 0, lds = 0;
        if ((e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
            (e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev)) != hipSuccess)
            return ladl::host_hipfail(e, "hipDeviceGetAttribute");
        d.num_cu = cu;
        d.lds_max = std::min<size_t>((size_t)lds, 160 * 1024);
        d.ptr = (unsigned char *)ptr;
    }
    out = d;
    return LADL_OK;
}

} // namespace

int ladl_solve_uniform_noalloc_f32(int32_t num_problems, int32_t n, int32_t p, int32_t path_len,
                                   const ladl_options *opt, const float *X, const float *y, const float *lambda,
                                   const float *b_init, float *b, float *obj, uint32_t *active, int32_t *zero_rows,
                                   int32_t *status, int32_t *iters, void *stream)
{
    using namespace ladl;
    if (num_problems < 1 || num_problems > LADL_NOALLOC_MAX_PROBLEMS)
        return host_fail(LADL_EUNSUPPORTED, "num_problems outside 1 .. LADL_NOALLOC_MAX_PROBLEMS");
    if (n < 1 || n > LADL_NOALLOC_MAX_ROWS) return host_fail(LADL_EUNSUPPORTED, "n outside 1 .. 1024");
    if (p < 1 || p > PMAX) return host_fail(LADL_EUNSUPPORTED, "p outside 1 .. 32");
    if (path_len < 1) return host_fail(LADL_EINVAL, "path_len must be >= 1");
    if ((int64_t)num_problems * path_len > (int64_t)INT32_MAX / 32)
        return host_fail(LADL_EUNSUPPORTED, "too many solve outputs");
    ladl_options o;
    ladl_default_options(&o);
    if (opt) o = *opt;
    int rc = host_check_options(&o);
    if (rc != LADL_OK) return rc;
    const bool quad = (o.flags & LADL_FLAG_QUADRATURE) != 0;
    if (!X || !y || !lambda || !b || !obj || !active || !zero_rows || !status)
        return host_fail(LADL_EINVAL, "a required device pointer is NULL");
    if (((uintptr_t)X | (uintptr_t)y | (uintptr_t)lambda | (uintptr_t)b_init | (uintptr_t)b | (uintptr_t)obj |
         (uintptr_t)active | (uintptr_t)zero_rows | (uintptr_t)status | (uintptr_t)iters) & 3)
        return host_fail(LADL_EINVAL, "device pointers must be 4-byte aligned");
    DeviceScratch d;
    if ((rc = device_scratch(d)) != LADL_OK) return rc;
    const int R = rows_per_lane(n);
    if (wave_lds_bytes(R, p, false, 0, 1) > d.lds_max)
        return host_fail(LADL_EUNSUPPORTED, "X of one problem does not fit the LDS of a CU");
    const int per_cu = std::max(1, wave_max_blocks_per_cu(R, p, false, false, 1, quad, 0));
    const int grid = (int)std::min<int64_t>(num_problems, (int64_t)per_cu * d.num_cu);
    hipStream_t s = (hipStream_t)stream;
    const int setup_blocks = std::min(1024, (num_problems + 1 + 255) / 256);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(setup_blocks), dim3(256), 0, s, d.ptr, (int)num_problems, (int)n,
                       (int)p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return host_hipfail(e, "scratch setup launch");
    SolveArgs a{};
    a.X = X;
    a.y = y;
    a.lam = lambda;
    a.b_init = b_init;
    a.row_off = (const int64_t *)(d.ptr + OFF_ROW);
    a.x_off = (const int64_t *)(d.ptr + OFF_XOFF);
    a.b_off = (const int64_t *)(d.ptr + OFF_BOFF);
    a.p_arr = (const int32_t *)(d.ptr + OFF_P);
    a.problem = nullptr;
    a.order = (const int32_t *)(d.ptr + OFF_ORDER);
    a.num_items = num_problems;
    a.path_len = path_len;
    a.t0 = 0;
    a.t1 = path_len;
    a.counter = (int32_t *)(d.ptr + OFF_COUNTER);
    a.b_out = b;
    a.obj_out = obj;
    a.active_out = active;
    a.zrows_out = zero_rows;
    a.status_out = status;
    a.iters_out = iters;
    a.gws = nullptr;
    a.gws_stride = 0;
    a.opt = host_dev_opt(o);
    a.pmax = p;
    a.nlds = p;
    e = launch_wave(R, false, false, 1, quad, a, grid, s);
    if (e != hipSuccess) return host_hipfail(e, "solve kernel launch");
    return LADL_OK;
}
