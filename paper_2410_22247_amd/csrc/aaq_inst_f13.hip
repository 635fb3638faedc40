// Kernel instantiations for complex64 amplitudes and tiles of 2^13 amplitudes.
#include "aaq_engine.h"

AAQ_INSTANTIATE_UNITS(float, 13, f13)
AAQ_INSTANTIATE_SWEEPS(float, 13, f13)
