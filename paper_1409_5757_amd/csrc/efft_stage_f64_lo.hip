// efft_stage_f64_lo.hip -- sub-FFT pass kernels for complex128 lines of 1 .. 256 points.
#include "efft_stage.hpp"

namespace efft {
EFFT_STAGE_LAUNCHER(launch_stage_f64_lo, double, 0, 8)
}  // namespace efft
