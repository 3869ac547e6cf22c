// 2D launchers at P = 6..10.
#define SHP_P2_LO 6
#define SHP_P2_HI 10
#include "shp_k_2d.inc"
