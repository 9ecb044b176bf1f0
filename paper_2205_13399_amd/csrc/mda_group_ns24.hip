// mda_group_ns24.hip -- the workgroup form built for 24 register slots per lane.
#define MDA_TILE 24
#include "mda_group_tile.h"
