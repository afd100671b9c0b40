// Instantiations of the persistent batch kernel for T = 15, 17 (one
// translation unit per group of window sides, so they compile in parallel).
#include "qfca_batch_impl.h"

QFCA_BATCH_INSTANTIATE(15)
QFCA_BATCH_INSTANTIATE(17)
