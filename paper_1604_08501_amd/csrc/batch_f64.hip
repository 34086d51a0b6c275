// Mixed-order batch kernel, double instantiation.
#define SEM_REAL double
#include "batch.inc"
