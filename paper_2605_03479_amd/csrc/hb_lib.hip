// The library is one translation unit: the single-case runtime and the
// batched form share the kernels defined in the headers.
#include "hb_runtime.hip"
#include "hb_batch.hip"
