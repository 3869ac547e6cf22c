// Whole-mesh launchers at P = 8.
#define SHP_P 8
#include "shp_k_mixed_p.inc"
