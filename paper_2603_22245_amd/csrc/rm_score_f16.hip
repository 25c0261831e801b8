// FP16 instantiations of the scoring kernel.  They live in a translation
// unit of their own so that they can be scheduled for instruction-level
// parallelism (the build passes LLVM's iterative-ilp machine scheduler for this
// file only): with it the compiler overlaps the next tile's B-fragment loads
// from LDS with the current tile's MFMAs.
#include "rm_score_kernel.h"

namespace rm {

namespace {

template <int KR>
hipError_t dispatch_f16(int read_tile, int kp, const ScoreLaunch& L, hipStream_t s) {
  if (read_tile == 256) {
    switch (kp) {
      case 8: return launch_persistent<RM_FP16, 2, 8, 32, 4, 1, KR>(L, s);
      case 16: return launch_persistent<RM_FP16, 2, 16, 32, 4, 1, KR>(L, s);
      // 32-key lists with a 16-slot buffer: 96 KB of lists leave room for
      // three ring stages
      default: return launch_persistent<RM_FP16, 2, 32, 48, 3, 1, KR>(L, s);
    }
  }
  switch (kp) {
    case 8: return launch_persistent<RM_FP16, 1, 8, 32, 4, 1, KR>(L, s);
    case 16: return launch_persistent<RM_FP16, 1, 16, 32, 4, 1, KR>(L, s);
    case 32: return launch_persistent<RM_FP16, 1, 32, 64, 4, 1, KR>(L, s);
    // 64-key lists with a 32-slot buffer: 96 KB of lists leave room for three
    // stages
    default: return launch_persistent<RM_FP16, 1, 64, 96, 3, 1, KR>(L, s);
  }
}

}  // namespace

hipError_t dispatch_score_f16(int read_tile, int kp, bool reduced, const ScoreLaunch& L,
                              hipStream_t s) {
  return reduced ? dispatch_f16<kRealReduced>(read_tile, kp, L, s)
                 : dispatch_f16<kReal>(read_tile, kp, L, s);
}

}  // namespace rm
