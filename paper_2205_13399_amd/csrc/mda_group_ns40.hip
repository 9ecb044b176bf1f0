// mda_group_ns40.hip -- the workgroup form built for 40 register slots per lane.
#define MDA_TILE 40
#include "mda_group_tile.h"
