// Whole-mesh launchers at P = 7.
#define SHP_P 7
#include "shp_k_mixed_p.inc"
