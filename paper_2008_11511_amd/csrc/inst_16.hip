// inst_16.hip - stack kernels and passes for 16 x 16 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(16)
