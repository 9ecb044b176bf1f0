// mda_group_ns32.hip -- the workgroup form built for 32 register slots per lane.
#define MDA_TILE 32
#include "mda_group_tile.h"
