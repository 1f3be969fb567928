// TI_n tiled step (sweep.h) for every compiled tile shape, FP32 and FP64.
#include "sweep.h"

namespace spfm {

template hipError_t launch_tiled_coupling<float, kLocal>(const float*, float*, const StepCoef<float>&,
                                                         int, int, const TileItem*, int,
                                                         const WallCoef<float>*, unsigned long long*, const CvFuse<float>*,
                                                         hipStream_t);
template hipError_t launch_tiled_coupling<double, kLocal>(const double*, double*,
                                                          const StepCoef<double>&, int, int,
                                                          const TileItem*, int,
                                                          const WallCoef<double>*, unsigned long long*, const CvFuse<double>*,
                                                          hipStream_t);

}  // namespace spfm
