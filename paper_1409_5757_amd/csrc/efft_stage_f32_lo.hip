// efft_stage_f32_lo.hip -- sub-FFT pass kernels for complex64 lines of 1 .. 256 points.
#include "efft_stage.hpp"

namespace efft {
EFFT_STAGE_LAUNCHER(launch_stage_f32_lo, float, 0, 8)
}  // namespace efft
