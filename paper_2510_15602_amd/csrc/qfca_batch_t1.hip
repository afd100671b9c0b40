// Instantiations of the persistent batch kernel for T = 3, 5, 7 (one
// translation unit per group of window sides, so they compile in parallel).
#include "qfca_batch_impl.h"

QFCA_BATCH_INSTANTIATE(3)
QFCA_BATCH_INSTANTIATE(5)
QFCA_BATCH_INSTANTIATE(7)
