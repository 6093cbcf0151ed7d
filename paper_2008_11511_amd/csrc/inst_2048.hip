// inst_2048.hip - stack kernels and passes for 2048 x 2048 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(2048)
