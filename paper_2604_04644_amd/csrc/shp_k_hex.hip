// Kernels of the hex shape.
#define SHP_SHAPE HEX
#define SHP_FN(name) name##hex
#include "shp_k_shape.inc"
