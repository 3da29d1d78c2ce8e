// mg_vcycle_static: one V-cycle whose workspace is a file-scope device array,
// for callers that cannot allocate device memory.  The plan is laid out on
// the host for this call and bound to the array with stream-ordered kernels
// (a fill kernel zeroes it, small kernels write the item tables); no
// hipMalloc, hipHostMalloc, hipFree, event or graph is created.
//
// Each device the library runs on holds its own copy of `scratch` until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy: its device address on the current device is taken once per device
// with hipGetSymbolAddress and used from then on.
#include "dmg_plan2d.hpp"
#include "dmg_plan3d.hpp"

#include <mutex>

using namespace dmg;

namespace {

constexpr size_t kScratchBytes = MG_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device (null until set up)

// The device address of `scratch` on device dev (the current device).
int scratch_on(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return MG_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MG_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MG_OK;
}

}  // namespace

extern "C" int mg_vcycle_static(int dim, int n, int precision, const double* p, int np, double* u, const double* f,
                                double* rel_res_before, void* hip_stream)
{
    if (!p || !u || !f || (dim != 2 && dim != 3)) return MG_ERR_ARG;
    if ((dim == 2 && np != 1) || (dim == 3 && np != 4)) return MG_ERR_ARG;
    for (int i = 0; i < np; i++)
        if (!(p[i] > 0 && p[i] < 1e6)) return MG_ERR_ARG;
    const int K = ilog2(n);
    if (K < 1 || (dim == 2 && K > 15) || (dim == 3 && K > 11)) return MG_ERR_SIZE;
    hipStream_t s = (hipStream_t)hip_stream;
    // argument and size errors are reported before any HIP call
    int dev = 0;
    void* ws = nullptr;
    if (dim == 2) {
        Plan2 P;
        int e = plan2_layout(P, 1, &n, precision, p[0], false);
        if (e) return e;
        if (P.total > kScratchBytes) return MG_ERR_SCRATCH;
        if (hipGetDevice(&dev) != hipSuccess) return MG_ERR_HIP;
        if ((e = scratch_on(dev, &ws)) || (e = plan2_bind_static(P, ws, s))) return e;
        return plan2_vcycle(P, &u, &f, rel_res_before);
    }
    Plan3 P;
    int e = plan3_layout(P, n, precision, p);
    if (e) return e;
    if (P.total > kScratchBytes) return MG_ERR_SCRATCH;
    if (hipGetDevice(&dev) != hipSuccess) return MG_ERR_HIP;
    if ((e = scratch_on(dev, &ws)) || (e = plan3_bind_static(P, ws, s))) return e;
    return plan3_vcycle(P, u, f, rel_res_before);
}
