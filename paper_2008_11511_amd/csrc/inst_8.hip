// inst_8.hip - stack kernels and passes for 8 x 8 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(8)
