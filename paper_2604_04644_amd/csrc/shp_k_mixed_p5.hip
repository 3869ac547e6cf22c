// Whole-mesh launchers at P = 5.
#define SHP_P 5
#include "shp_k_mixed_p.inc"
