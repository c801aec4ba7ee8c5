// depths.hpp -- which (storage type, stencil) pairs are compiled and how deep
// their fused kernels go.  Single table read by the dispatchers and the planner.
#pragma once
#include "launch.hpp"

namespace so2dr {

// rows: so2dr_dtype F32, F64, BF16, F16; columns: StencilId
constexpr int kMaxDepth[4][ST_COUNT] = {
    /* F32  */ {8, 8, 4, 4, 4, 4, 2, 4},
    /* F64  */ {4, 4, 2, 2, 2, 2, 2, 2},
    /* BF16 */ {8, 8, 4, 4, 4, 4, 2, 4},
    /* F16  */ {8, 8, 4, 4, 4, 4, 2, 4},
};

}  // namespace so2dr
