// inst_128.hip - stack kernels and passes for 128 x 128 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(128)
