// Kernel instantiations for complex64 amplitudes and tiles of 2^10 amplitudes.
#include "aaq_engine.h"

AAQ_INSTANTIATE_UNITS(float, 10, f10)
