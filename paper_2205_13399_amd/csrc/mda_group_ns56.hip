// mda_group_ns56.hip -- the workgroup form built for 56 register slots per lane.
#define MDA_TILE 56
#include "mda_group_tile.h"
