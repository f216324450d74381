// Persistent merge kernels instantiated for int32_t keys (see mp_stream_impl.h).
#include "mp_stream_impl.h"

MP_STREAM_INSTANTIATE(int32_t)
