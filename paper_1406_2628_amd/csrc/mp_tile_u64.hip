// Per-tile merge kernels for uint64_t keys.
#include "mp_tile_impl.h"
MP_TILE_INSTANTIATE(uint64_t)
