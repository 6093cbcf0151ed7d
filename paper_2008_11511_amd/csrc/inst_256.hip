// inst_256.hip - stack kernels and passes for 256 x 256 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(256)
