// mda_group_ns8.hip -- the workgroup form built for 8 register slots per lane.
#define MDA_TILE 8
#include "mda_group_tile.h"
