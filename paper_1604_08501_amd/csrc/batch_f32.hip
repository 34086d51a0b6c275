// Mixed-order batch kernel, float instantiation.
#define SEM_REAL float
#include "batch.inc"
