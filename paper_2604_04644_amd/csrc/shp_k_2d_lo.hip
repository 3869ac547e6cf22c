// 2D launchers at P = 1..5.
#define SHP_P2_LO 1
#define SHP_P2_HI 5
#include "shp_k_2d.inc"
