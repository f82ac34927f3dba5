// snap_static.hip -- the static device workspace of snap_compute_noalloc:
// one file-scope array per GPU, held until the process ends, so that the
// evaluation can run where no device memory may be allocated.
#include <mutex>

#include "snap_kernels.hpp"

namespace snapmi {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

__global__ void k_zero_cols(double2 *__restrict__ p, int rows, int npad, int n)
{
    // p[r * npad + a] = 0 for a in [n, npad): the padding atoms of an
    // element-major array
    const int w = npad - n;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)rows * w) return;
    const int r = (int)(k / w), a = n + (int)(k - (size_t)r * w);
    p[(size_t)r * npad + a] = make_double2(0.0, 0.0);
}

__global__ void k_zero(double2 *__restrict__ p, size_t count)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = make_double2(0.0, 0.0);
}

}  // namespace

// In host code this name stands for the array, not its device address: the
// address comes from hipGetSymbolAddress, looked up once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t static_scratch_bytes() { return kScratchBytes; }

hipError_t static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

hipError_t launch_zero_padding(double2 *U, int nfull, double2 *Y, int nhalf, int n, int npad,
                               hipStream_t s)
{
    if (npad > n) {
        const size_t cu = (size_t)nfull * (npad - n);
        hipLaunchKernelGGL(k_zero_cols, dim3((unsigned)((cu + 255) / 256)), dim3(256), 0, s, U,
                           nfull, npad, n);
        // Y is atom-major: the padding atoms' rows are one contiguous range
        const size_t cy = (size_t)nhalf * (npad - n);
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((cy + 255) / 256)), dim3(256), 0, s,
                           Y + (size_t)n * nhalf, cy);
    }
    return hipGetLastError();
}

}  // namespace snapmi
