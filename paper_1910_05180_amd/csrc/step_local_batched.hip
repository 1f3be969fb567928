// TI_n batched step (sweep.h) for every compiled tile shape.
#include "sweep.h"

namespace spfm {

template hipError_t launch_batched_coupling<kLocal>(const float*, float*, const StepCoef<float>*,
                                                    const int64_t*, int, int, const TileItem*, int,
                                                    const WallCoef<float>*, hipStream_t);

}  // namespace spfm
