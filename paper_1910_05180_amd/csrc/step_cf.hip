// Continuum-field control (h3, h5, h_Abel) tiled and batched steps (sweep.h)
// for every compiled tile shape.
#include "sweep.h"

namespace spfm {

#define SPFM_CF_INSTANCES(C_)                                                                      \
    template hipError_t launch_tiled_coupling<float, C_>(const float*, float*,                      \
                                                         const StepCoef<float>&, int, int,          \
                                                         const TileItem*, int,                      \
                                                         const WallCoef<float>*,                    \
                                                         unsigned long long*,                       \
                                                         const CvFuse<float>*, hipStream_t);        \
    template hipError_t launch_tiled_coupling<double, C_>(const double*, double*,                   \
                                                          const StepCoef<double>&, int, int,        \
                                                          const TileItem*, int,                     \
                                                          const WallCoef<double>*,                  \
                                                          unsigned long long*,                      \
                                                          const CvFuse<double>*, hipStream_t);      \
    template hipError_t launch_batched_coupling<C_>(const float*, float*, const StepCoef<float>*,   \
                                                    const int64_t*, int, int, const TileItem*, int, \
                                                    const WallCoef<float>*, hipStream_t);
SPFM_CF_INSTANCES(kCF)
SPFM_CF_INSTANCES(kCF5)
SPFM_CF_INSTANCES(kCFAbel)
#undef SPFM_CF_INSTANCES

}  // namespace spfm
