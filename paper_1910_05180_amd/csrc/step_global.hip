// TI_<hkl> tiled and batched steps (sweep.h) for every compiled tile shape.
#include "sweep.h"

namespace spfm {

template hipError_t launch_tiled_coupling<float, kGlobal>(const float*, float*, const StepCoef<float>&,
                                                          int, int, const TileItem*, int,
                                                          const WallCoef<float>*, unsigned long long*, const CvFuse<float>*,
                                                         hipStream_t);
template hipError_t launch_tiled_coupling<double, kGlobal>(const double*, double*,
                                                           const StepCoef<double>&, int, int,
                                                           const TileItem*, int,
                                                           const WallCoef<double>*, unsigned long long*, const CvFuse<double>*,
                                                          hipStream_t);
template hipError_t launch_batched_coupling<kGlobal>(const float*, float*, const StepCoef<float>*,
                                                     const int64_t*, int, int, const TileItem*, int,
                                                     const WallCoef<float>*, hipStream_t);

}  // namespace spfm
