// fv_stage_inst.hip -- the stage kernels of one precision and model (every
// limiter, reconstruction and viscosity-law variant), compiled once per
// (FV_REAL, FV_MODEL) pair given on the command line.
#include "fv_stage.h"

#if !defined(FV_REAL) || !defined(FV_MODEL)
#error "compile with -DFV_REAL=double|float -DFV_MODEL=EULER|NS|DIM"
#endif

namespace fv {
template hipError_t launch_model<FV_REAL, FV_MODEL>(const StageArgs<FV_REAL>&, const LaunchGeom&, hipStream_t);
}  // namespace fv
