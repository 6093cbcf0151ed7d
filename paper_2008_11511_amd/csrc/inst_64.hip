// inst_64.hip - stack kernels and passes for 64 x 64 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(64)
