// tri_device.h -- device helpers shared by the libtri kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "tri_internal.h"

namespace tri {

typedef double v2d __attribute__((ext_vector_type(2)));   // 16-byte vector access

// Global-address-space views of table and field pointers.  The solve bodies
// load through these, so the compiler emits global (and, for uniform
// addresses, scalar) loads even where the pointer was read from memory, as
// in the batched launches, rather than flat ones.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) int gint;

// ===========================================================================
// Reduced-system evaluation shared by the solve kernels: the left and right
// interface unknowns of partition r from the tips of its line.
// tip(q): q = 2*partition (first row) or 2*partition + 1 (last row).
// ===========================================================================
template <int METHOD, typename ItPtr, typename TipFn>
__device__ __forceinline__ void interface_unknowns(ItPtr it, int r, int P, int periodic, TipFn tip, double &yl,
                                                   double &yr)
{
    yl = 0.0;
    yr = 0.0;
    const bool has_l = (r > 0) || periodic;
    const bool has_r = (r < P - 1) || periodic;
    const int rowlen = 2 * P;
    if (METHOD == TRI_PDD) {
        if (has_l) {
            const int L = (r > 0) ? r - 1 : P - 1;
            yl = it[2 * L + 1] * tip(2 * L + 1) + it[2 * r] * tip(2 * r);
        }
        if (has_r) {
            const int R = (r < P - 1) ? r + 1 : 0;
            yr = it[rowlen + 2 * R] * tip(2 * R) + it[rowlen + 2 * r + 1] * tip(2 * r + 1);
        }
    } else {
        const int q0 = periodic ? 0 : 1;
        const int q1 = periodic ? rowlen : rowlen - 1;
        if (has_l)
            for (int q = q0; q < q1; ++q) yl += it[q] * tip(q);
        if (has_r)
            for (int q = q0; q < q1; ++q) yr += it[rowlen + q] * tip(q);
    }
}

}  // namespace tri
