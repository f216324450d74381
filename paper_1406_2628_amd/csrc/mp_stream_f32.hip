// Persistent merge kernels instantiated for float keys (see mp_stream_impl.h).
#include "mp_stream_impl.h"

MP_STREAM_INSTANTIATE(float)
