// Extended single-order kernels (tracers, direction subsets, Nq up to 16), float instantiation.
#define SEM_REAL float
#include "ext.inc"
