// efft_stage_f64_hi.hip -- sub-FFT pass kernels for complex128 lines of 512 .. 4096 points.
#include "efft_stage.hpp"

namespace efft {
EFFT_STAGE_LAUNCHER(launch_stage_f64_hi, double, 9, 12)
}  // namespace efft
