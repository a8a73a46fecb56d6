// fv_stage_launch.hip -- dispatch of the stage kernels by model and the
// batched (many-problem) stage kernels.
#include "fv_stage.h"

namespace fv {

// the kernel families (and the batched kernels) live in fv_stage_inst.hip objects
#define FV_EXTERN_BATCH(R, M, REC)                                                                           \
    extern template hipError_t launch_batch_rec<R, M, REC>(bool, int, const StageArgs<R>*, const int*, const int*, \
                                                           int, hipStream_t);
#define FV_EXTERN_REC(R, M)                                                                                    \
    FV_EXTERN_BATCH(R, M, REC_WENO_PRIM)                                                                       \
    FV_EXTERN_BATCH(R, M, REC_WENO_CHAR)                                                                       \
    FV_EXTERN_BATCH(R, M, REC_TENO_PRIM)                                                                       \
    FV_EXTERN_BATCH(R, M, REC_TENO_CHAR)                                                                       \
    extern template hipError_t launch_rec<R, M, REC_WENO_PRIM>(const StageArgs<R>&, const LaunchGeom&, hipStream_t); \
    extern template hipError_t launch_rec<R, M, REC_WENO_CHAR>(const StageArgs<R>&, const LaunchGeom&, hipStream_t); \
    extern template hipError_t launch_rec<R, M, REC_TENO_PRIM>(const StageArgs<R>&, const LaunchGeom&, hipStream_t); \
    extern template hipError_t launch_rec<R, M, REC_TENO_CHAR>(const StageArgs<R>&, const LaunchGeom&, hipStream_t);
FV_EXTERN_REC(double, EULER)
FV_EXTERN_REC(double, NS)
FV_EXTERN_REC(double, DIM)
FV_EXTERN_REC(float, EULER)
FV_EXTERN_REC(float, NS)
FV_EXTERN_REC(float, DIM)
#undef FV_EXTERN_REC
#undef FV_EXTERN_BATCH

template hipError_t launch_batch_stage<double>(int, int, bool, int, const StageArgs<double>*, const int*, const int*,
                                                int, hipStream_t);
template hipError_t launch_batch_stage<float>(int, int, bool, int, const StageArgs<float>*, const int*, const int*, int,
                                               hipStream_t);

template hipError_t launch_stage<double>(int, const StageArgs<double>&, const LaunchGeom&, hipStream_t);
template hipError_t launch_stage<float>(int, const StageArgs<float>&, const LaunchGeom&, hipStream_t);

}  // namespace fv
