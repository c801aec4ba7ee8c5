// rates.hpp -- measured update rates of the fused-step kernels on MI355X,
// read by the planner (automatic fused depth) and the cost model.
//
// G cell-updates/s (output cells x fused levels per second) of one launch by
// storage type, stencil id and depth 1..8 (0 = depth not built), measured
// with so2dr_kernel_bench (`bench.py --kernel-rates --grid ...`) over an
// interior chunk of 64 output planes of a 2048 x 1024 plane in 3D and 1200
// output rows of 38400 cells in 2D.  The 2D chunks of 16-bit storage fit
// the 256 MiB last-level cache in part, which their rates include.
#pragma once

namespace so2dr {

// rows: so2dr_dtype F32, F64, BF16, F16; then StencilId; then depth - 1
constexpr double kRate[4][8][8] = {
    {
        // F32
        {583, 1122, 1619, 2105, 2379, 2732, 2927, 3005},  // 2D star r1
        {551, 1072, 1558, 1942, 1997, 2017, 2034, 2034},  // 2D box r1
        {555, 787, 791, 807, 0, 0, 0, 0},                 // 2D box r2
        {424, 401, 394, 393, 0, 0, 0, 0},                 // 2D box r3
        {236, 225, 217, 200, 0, 0, 0, 0},                 // 2D box r4
        {538, 1149, 1535, 1308, 0, 0, 0, 0},              // 3D star r1
        {557, 884, 0, 0, 0, 0, 0, 0},                     // 3D star r2
        {512, 792, 675, 530, 0, 0, 0, 0},                 // 3D box r1
    },
    {
        // F64
        {264, 515, 759, 972, 0, 0, 0, 0},
        {261, 501, 738, 966, 0, 0, 0, 0},
        {258, 494, 0, 0, 0, 0, 0, 0},
        {230, 239, 0, 0, 0, 0, 0, 0},
        {124, 117, 0, 0, 0, 0, 0, 0},
        {260, 533, 0, 0, 0, 0, 0, 0},
        {270, 248, 0, 0, 0, 0, 0, 0},
        {254, 511, 0, 0, 0, 0, 0, 0},
    },
    {
        // BF16
        {1538, 2584, 2846, 2923, 2700, 2729, 2744, 2659},
        {1423, 1950, 1993, 2019, 1899, 1914, 1906, 1911},
        {773, 832, 802, 799, 0, 0, 0, 0},
        {447, 413, 403, 384, 0, 0, 0, 0},
        {234, 224, 217, 198, 0, 0, 0, 0},
        {1004, 1330, 1486, 1234, 0, 0, 0, 0},
        {776, 914, 0, 0, 0, 0, 0, 0},
        {555, 802, 717, 514, 0, 0, 0, 0},
    },
    {
        // F16
        {1483, 2390, 2473, 2510, 2526, 2510, 2532, 2486},
        {1396, 1822, 1924, 1974, 1899, 1897, 1915, 1873},
        {729, 788, 772, 783, 0, 0, 0, 0},
        {427, 395, 386, 373, 0, 0, 0, 0},
        {228, 219, 214, 195, 0, 0, 0, 0},
        {993, 1290, 1414, 1162, 0, 0, 0, 0},
        {710, 876, 0, 0, 0, 0, 0, 0},
        {586, 769, 698, 510, 0, 0, 0, 0},
    },
};

// Measured rate of a launch fusing `levels` steps (0 when not measured or
// not built).
constexpr double kernel_rate(int dtype, int stencil, int levels) {
  return dtype >= 0 && dtype < 4 && stencil >= 0 && stencil < 8 && levels >= 1 && levels <= 8
             ? kRate[dtype][stencil][levels - 1]
             : 0.0;
}

// Fused depth for a plan that leaves k_on to the library: the shallowest
// depth (at most max_depth) within 3 % of the best measured rate -- deeper
// launches recompute more tile edges for little gain.
constexpr int preferred_depth(int dtype, int stencil, int max_depth) {
  double best = 0.0;
  for (int k = 1; k <= max_depth && k <= 8; ++k)
    if (kernel_rate(dtype, stencil, k) > best) best = kernel_rate(dtype, stencil, k);
  for (int k = 1; k <= max_depth && k <= 8; ++k)
    if (kernel_rate(dtype, stencil, k) >= 0.97 * best && best > 0.0) return k;
  return 1;
}

}  // namespace so2dr
