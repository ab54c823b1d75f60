// Host stand-ins for the HIP runtime calls and kernel launchers that libtri's
// API layer (tri_api.hip) uses, so that the layer builds and runs on a CPU
// under AddressSanitizer/UndefinedBehaviorSanitizer.  No kernel runs: every
// launcher only counts the launch.  "Device" allocations are zero-filled host
// memory; the counters let the driver check that a call launched nothing or
// allocated nothing.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <initializer_list>
#include <cstring>

#include "tri_internal.h"
#include "tri_ns.h"

int g_launches = 0;      // kernel launches since start
int g_mallocs = 0;       // hipMalloc calls since start
int g_frees = 0;
int g_syncs = 0;         // stream/event synchronisations
int g_symbol_lookups = 0;

struct ihipStream_t { int dummy; };
struct ihipEvent_t { int dummy; };
struct ihipGraph { int dummy; };
struct hipGraphExec { int dummy; };

hipError_t hipGetDeviceCount(int *count) { *count = 1; return hipSuccess; }
hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipMalloc(void **p, size_t bytes)
{
    ++g_mallocs;
    const size_t n = ((bytes ? bytes : 1) + 255) / 256 * 256;
    *p = std::aligned_alloc(256, n);
    if (!*p) return hipErrorOutOfMemory;
    std::memset(*p, 0, n);
    return hipSuccess;
}
hipError_t hipFree(void *p) { ++g_frees; std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind)
{
    std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemset(void *dst, int value, size_t bytes) { std::memset(dst, value, bytes); return hipSuccess; }
hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t) { return hipMemset(dst, value, bytes); }
hipError_t hipStreamSynchronize(hipStream_t) { ++g_syncs; return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new ihipStream_t(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = new ihipGraph(); return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, hipGraphNode_t *, char *, size_t)
{
    *e = new hipGraphExec();
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { ++g_syncs; return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
hipError_t hipGetSymbolAddress(void **p, const void *symbol)
{
    ++g_symbol_lookups;
    *p = const_cast<void *>(symbol);
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "stub"; }

namespace tri {

static hipError_t counted() { ++g_launches; return hipSuccess; }

hipError_t launch_factor(const MatSrc &, const Tables &, int *, hipStream_t) { return counted(); }
hipError_t launch_strided(const SolveArgs &, int, int, hipStream_t) { return counted(); }
bool strided_acc_supported(int method, int chunk_max) { return method == 0 && chunk_max <= 24; }
bool strided2_acc_supported(int method, int chunk_max) { return method == 0 && chunk_max == 24; }
size_t strided_lds_bytes(const SolveArgs &) { return 4096; }
hipError_t launch_strided2(const SolveArgs &, int, int, hipStream_t) { return counted(); }
hipError_t launch_strided_batch(const BatchEntry *, int, int64_t, int, int, int, bool, size_t, hipStream_t)
{
    return counted();
}
hipError_t launch_contig(const SolveArgs &, int, hipStream_t) { return counted(); }
hipError_t launch_level(const LevelEntry *, int, int64_t, size_t, hipStream_t) { return counted(); }
hipError_t launch_contig_staged(const SolveArgs &, int, int, hipStream_t) { return counted(); }
size_t contig_staged_lds_bytes(const SolveArgs &) { return 4096; }
int contig_staged_grid(const SolveArgs &, int) { return 256; }
hipError_t launch_contig_reg(const SolveArgs &, int, int, hipStream_t) { return counted(); }
size_t contig_reg_lds_bytes(const SolveArgs &) { return 4096; }
int contig_reg_grid(const SolveArgs &, int) { return 256; }
hipError_t launch_general(const GeneralArgs &, int, hipStream_t) { return counted(); }
hipError_t launch_strided_refine(const SolveArgs &, const RefineArgs &, int, int, hipStream_t) { return counted(); }
size_t strided_refine_lds_bytes(const SolveArgs &) { return 4096; }
hipError_t launch_strided_refine_batch(const BatchEntry *, int, int64_t, int, int, int, bool, size_t, hipStream_t)
{
    return counted();
}
hipError_t launch_contig_refine(const SolveArgs &, const RefineArgs &, int, int, hipStream_t) { return counted(); }
size_t contig_refine_lds_bytes(const SolveArgs &) { return 4096; }
int contig_refine_grid(const SolveArgs &, int) { return 256; }
hipError_t launch_general_refine(const GeneralArgs &, const RefineArgs &, int, hipStream_t) { return counted(); }
hipError_t launch_reset_counters(int *, unsigned long long *, hipStream_t) { return counted(); }
hipError_t launch_stream_copy(double *, const double *, int64_t, hipStream_t) { return counted(); }
hipError_t launch_fft(const FftArgs &, int, hipStream_t) { return counted(); }
hipError_t launch_grad_y(double *, const double *, const double *, int64_t, int64_t, int64_t, hipStream_t)
{
    return counted();
}
hipError_t launch_dct(const DctArgs &, bool, hipStream_t) { return counted(); }
hipError_t launch_grad_xy(double *, double *, const double *, const double *, double, int64_t, int64_t, int64_t,
                          hipStream_t)
{
    return counted();
}

hipError_t launch_ns_rhs(const NsRhsArgs &, hipStream_t) { return counted(); }
hipError_t launch_ns_update(double *, double *, double *, const double *, const double *, const double *, int64_t,
                            int64_t, int64_t, hipStream_t)
{
    return counted();
}
hipError_t launch_ns_pressure(double *, const double *, double, int64_t, hipStream_t) { return counted(); }
hipError_t launch_grad_xy_pressure(double *, double *, const double *, const double *, double, int64_t, int64_t,
                                   int64_t, double *, double, hipStream_t)
{
    return counted();
}

// Transform shapes: the documented contract (the real ones live with the
// transform kernels): N = 2^a 3^b 5^c within the limit.
static bool smooth(int64_t N, FftShape &S)
{
    int64_t r = N;
    S = FftShape{};
    S.M = (int)N;
    for (int f : {4, 2, 3, 5})
        while (r % f == 0 && S.npass < kFftMaxPasses) {
            S.radix[S.npass++] = f;
            r /= f;
        }
    return r == 1;
}
bool fft_shape(int64_t Nz, FftShape &S)
{
    if (Nz < 2 || Nz % 2) return false;
    return Nz / 2 <= kFftMaxM && smooth(Nz / 2, S);
}
bool dct_shape(int64_t N, FftShape &S)
{
    if (N < 2 || N % 2 || N > kDctMaxN) return false;
    return smooth(N, S);
}

}  // namespace tri
