// mda_generic_k4.hip -- the K-objective kernels for K = 4 (every slot count).
#define MDA_GK 4
#include "mda_generic_tile.h"
