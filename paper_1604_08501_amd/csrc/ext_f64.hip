// Extended single-order kernels (tracers, direction subsets, Nq up to 16), double instantiation.
#define SEM_REAL double
#include "ext.inc"
