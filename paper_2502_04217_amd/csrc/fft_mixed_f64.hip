// FP64 pencil-FFT passes at the grid extents with odd factors 3, 5 and 7
// (CSIPM_MIXED_LENGTHS): the kernels of the power-of-two lengths with
// odd-radix Stockham stages.  One translation unit per precision so that
// the instantiations compile in parallel.
#include "fft_kernels.h"

namespace csipm {
namespace fftk {

CSIPM_MIXED_INSTANCES(, double)
CSIPM_MIXED_INST12(, double, 1, -1, EpiR)

}  // namespace fftk
}  // namespace csipm
