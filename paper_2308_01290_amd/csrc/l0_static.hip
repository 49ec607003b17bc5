// Allocation-free gradient-L0 step: the unit-weight path of dect_l0_step (the
// FFT closed form of eq. (5)-(9)) with its complex scratch in a file-scope
// device array instead of a workspace.  For callers that cannot allocate
// device memory (graph capture, serving loops).
//
// The array is one per GPU, held until the process ends; every call on a GPU
// uses it, so calls that overlap on one GPU race.  Each call overwrites every
// scratch value it reads (the row pass writes the whole batch*n_y*n_x plane
// before the column pass reads it), so nothing has to start at zero.
#include <mutex>
#include <vector>

#include "dect_internal.h"

namespace dect {

// complex scratch values (float2): batch * n_y * n_x at most, 16 MiB
constexpr size_t kL0StaticValues = (size_t)1 << 21;
static __device__ __align__(256) float2 scratch[kL0StaticValues];

// device address of `scratch` on each GPU, taken once per device with that
// device current (the host-side name is not a device address)
static std::mutex g_scratch_mu;
static std::vector<float2*> g_scratch_ptr;

static int scratch_address(float2** out) {
    int dev = 0;
    DECT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DECT_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float2*>(p);
    }
    *out = g_scratch_ptr[dev];
    return DECT_OK;
}

}  // namespace dect

using namespace dect;

extern "C" {

size_t dect_l0_step_static_max_values(void) { return kL0StaticValues; }

int dect_l0_step_static(const float* g_tilde, float* g, float* h_out, float* v_out, int32_t n_y,
                        int32_t n_x, int32_t batch, double lambda, double beta, hipStream_t st) {
    if (batch < 0) return fail(DECT_EINVAL, "batch must be >= 0");
    if (batch == 0) return DECT_OK;
    if (!g_tilde || !g) return fail(DECT_EINVAL, "dect_l0_step_static: NULL g_tilde or g");
    if (!fft_size_ok(n_x) || !fft_size_ok(n_y))
        return fail(DECT_EINVAL,
                    "dect_l0_step_static: n_x=%d n_y=%d must be 2^a*3^b (b<=1) in [8, 1024]", n_x,
                    n_y);
    if (!(lambda >= 0) || !(beta > 0)) return fail(DECT_EINVAL, "need lambda >= 0 and beta > 0");
    const size_t values = (size_t)batch * (size_t)n_y * (size_t)n_x;
    if (values > kL0StaticValues)
        return fail(DECT_EINVAL,
                    "dect_l0_step_static: batch*n_y*n_x = %zu exceeds the static scratch of %zu "
                    "values (use dect_l0_step with a workspace)",
                    values, kL0StaticValues);
    float2* fft = nullptr;
    if (int rc = scratch_address(&fft)) return rc;
    return l0_fft_step(g_tilde, g, h_out, v_out, n_y, n_x, batch, lambda, beta, fft, st);
}

}  // extern "C"
