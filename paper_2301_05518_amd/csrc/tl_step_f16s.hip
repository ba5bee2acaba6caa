// Smearing step kernels stored in F16S: every link form (two-links or one-links, 18 or 12 reals).
#include "tl_step.h"

namespace tl {

hipError_t launch_step_f16s(int form, int width, const StepConfig& cfg, const StepGroup* groups, int n_groups,
                          int tile_base, int n_tiles, const char* in, char* out, double alpha, double beta,
                          int64_t lds, hipStream_t stream) {
  return launch_step_both<F16S>(form, width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds,
                          stream);
}

hipError_t step_attributes_f16s() { return step_attributes_both<F16S>(); }

}  // namespace tl
