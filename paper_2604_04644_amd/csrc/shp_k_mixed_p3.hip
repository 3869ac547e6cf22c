// Whole-mesh launchers at P = 3.
#define SHP_P 3
#include "shp_k_mixed_p.inc"
