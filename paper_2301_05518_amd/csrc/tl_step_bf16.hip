// Smearing step kernels stored in BF16: every link form (two-links or one-links, 18 or 12 reals).
#include "tl_step.h"

namespace tl {

hipError_t launch_step_bf16(int form, int width, const StepConfig& cfg, const StepGroup* groups, int n_groups,
                          int tile_base, int n_tiles, const char* in, char* out, double alpha, double beta,
                          int64_t lds, hipStream_t stream) {
  return launch_step_both<BF16>(form, width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds,
                          stream);
}

hipError_t step_attributes_bf16() { return step_attributes_both<BF16>(); }

}  // namespace tl
