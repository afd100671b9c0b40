// Instantiations of the persistent batch kernel for T = 27, 29 (one
// translation unit per group of window sides, so they compile in parallel).
#include "qfca_batch_impl.h"

QFCA_BATCH_INSTANTIATE(27)
QFCA_BATCH_INSTANTIATE(29)
