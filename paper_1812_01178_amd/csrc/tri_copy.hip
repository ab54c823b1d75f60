// tri_copy.hip -- reference copy for bandwidth fractions (not a step of the
// method).  A solve moves each unknown from HBM once and back once, so the
// bandwidth a plain copy attains on the same device is the attainable bound
// of every solve kernel; this is that copy, written the way the fastest
// streaming copy on gfx950 is: one pass (one 16-byte vector per lane, no
// grid-stride loop), non-temporal loads and stores.
#include "tri_internal.h"

namespace tri {
namespace {

typedef double v2d __attribute__((ext_vector_type(2)));
constexpr int kCopyBlock = 256;

// Thread i copies the pair (2i, 2i+1); when n is odd, thread n/2 copies the
// last element alone (dst may equal src: each element is read and written
// by the same lane).  The grid covers ceil(n/2) threads exactly, rounded up
// to whole blocks; excess lanes return.
__global__ void __launch_bounds__(kCopyBlock) k_stream_copy(double *dst, const double *src,
                                                             int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kCopyBlock + threadIdx.x;
    const int64_t pairs = n >> 1;
    if (i < pairs) {
        const v2d v = __builtin_nontemporal_load((const v2d *)src + i);
        __builtin_nontemporal_store(v, (v2d *)dst + i);
    } else if (i == pairs && (n & 1)) {
        dst[n - 1] = src[n - 1];
    }
}

}  // namespace

hipError_t launch_stream_copy(double *dst, const double *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t threads = (n + 1) >> 1;
    const int64_t blocks = (threads + kCopyBlock - 1) / kCopyBlock;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kCopyBlock), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace tri
