// tri_contig_reg.hip -- contiguous-row partitioned solve with the shared
// matrix's factors held in registers, as a persistent kernel: one line per
// workgroup at a time, several small workgroups resident per CU so that one
// workgroup's barriers and memory waits overlap the others' work (the solve
// itself is contig_reg_solve in tri_contig_reg.h).
#include <hip/hip_runtime.h>

#include "tri_contig_reg.h"

namespace tri {

template <int C, int METHOD>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(C == 8 ? 2 : 4)))
k_contig_reg(const SolveArgs A)
{
    extern __shared__ double lds[];
    contig_reg_solve<C, METHOD>(A, blockIdx.x, gridDim.x, 0, (int)threadIdx.x, lds);
}

size_t contig_reg_lds_bytes(const SolveArgs &a)
{
    return sizeof(double) * ((size_t)2 * (a.C / 2) * a.stage_stride + 2 * (size_t)a.P + 4 * (size_t)a.P * a.P);
}

template <int C, int METHOD>
static hipError_t launch_contig_reg_t(const SolveArgs &a, int grid, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>(std::max(grid, 1), a.nlines);
    hipLaunchKernelGGL((k_contig_reg<C, METHOD>), dim3((unsigned)blocks), dim3(a.LL), contig_reg_lds_bytes(a), s, a);
    return hipGetLastError();
}

template <int C, int METHOD>
static int contig_reg_grid_t(const SolveArgs &a)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_contig_reg<C, METHOD>),
                                                     a.LL, contig_reg_lds_bytes(a)) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return std::max(1, per_cu) * cus;
}

int contig_reg_grid(const SolveArgs &a, int method)
{
    const bool pdd = method == TRI_PDD;
    if (a.C == 4) return pdd ? contig_reg_grid_t<4, TRI_PDD>(a) : contig_reg_grid_t<4, TRI_PPT>(a);
    if (a.C == 8) return pdd ? contig_reg_grid_t<8, TRI_PDD>(a) : contig_reg_grid_t<8, TRI_PPT>(a);
    return 0;
}

hipError_t launch_contig_reg(const SolveArgs &a, int method, int grid, hipStream_t s)
{
    if (a.C == 4)
        return method == TRI_PDD ? launch_contig_reg_t<4, TRI_PDD>(a, grid, s)
                                 : launch_contig_reg_t<4, TRI_PPT>(a, grid, s);
    if (a.C == 8)
        return method == TRI_PDD ? launch_contig_reg_t<8, TRI_PDD>(a, grid, s)
                                 : launch_contig_reg_t<8, TRI_PPT>(a, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace tri
