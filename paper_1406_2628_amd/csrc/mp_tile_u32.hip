// Per-tile merge kernels for uint32_t keys.
#include "mp_tile_impl.h"
MP_TILE_INSTANTIATE(uint32_t)
