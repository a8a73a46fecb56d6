// fv_stage_inst.hip -- the stage kernels of one precision, model and
// reconstruction (every limiter and viscosity variant), compiled once per
// (FV_REAL, FV_MODEL, FV_REC) triple given on the command line.
#include "fv_stage.h"

#if !defined(FV_REAL) || !defined(FV_MODEL) || !defined(FV_REC)
#error "compile with -DFV_REAL=double|float -DFV_MODEL=EULER|NS|DIM -DFV_REC=0..3"
#endif

namespace fv {
template hipError_t launch_rec<FV_REAL, FV_MODEL, FV_REC>(const StageArgs<FV_REAL>&, const LaunchGeom&, hipStream_t);
// the batched kernels of the same family share its body and compile options
template hipError_t launch_batch_rec<FV_REAL, FV_MODEL, FV_REC>(bool, int, const StageArgs<FV_REAL>*, const int*,
                                                                const int*, int, hipStream_t);
}  // namespace fv
