// inst_512.hip - stack kernels and passes for 512 x 512 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(512)
