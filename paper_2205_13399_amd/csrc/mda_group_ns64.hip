// mda_group_ns64.hip -- the workgroup form built for 64 register slots per lane.
#define MDA_TILE 64
#include "mda_group_tile.h"
