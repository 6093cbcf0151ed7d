// inst_1024.hip - stack kernels and passes for 1024 x 1024 frames.
#include "passes.hpp"

PTYCHO_DEFINE_PASSES(1024)
