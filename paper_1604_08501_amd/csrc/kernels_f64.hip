// Single-order kernels, double instantiation.
#define SEM_REAL double
#include "kernels.inc"
