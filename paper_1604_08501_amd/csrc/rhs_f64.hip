// Whole-rate (volume + surface) kernel, double instantiation.
#define SEM_REAL double
#include "rhs.inc"
