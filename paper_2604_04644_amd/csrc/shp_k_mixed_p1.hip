// Whole-mesh launchers at P = 1.
#define SHP_P 1
#include "shp_k_mixed_p.inc"
