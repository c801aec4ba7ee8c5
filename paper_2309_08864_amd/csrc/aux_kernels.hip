// aux_kernels.hip -- small device helpers shared by the executor (reserved
// for the adjoint's FP64 reductions).
#include <hip/hip_runtime.h>
