// inst_32.hip - stack kernels and passes for 32 x 32 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(32)
