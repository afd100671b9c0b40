// Instantiations of the persistent batch kernel for T = 9, 11, 13 (one
// translation unit per group of window sides, so they compile in parallel).
#include "qfca_batch_impl.h"

QFCA_BATCH_INSTANTIATE(9)
QFCA_BATCH_INSTANTIATE(11)
QFCA_BATCH_INSTANTIATE(13)
