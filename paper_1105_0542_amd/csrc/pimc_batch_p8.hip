// Launch-shape variants of the batched kernel at level p = 8 (see pimc_batch.hpp).
#include "pimc_batch.hpp"

namespace pimc {
PIMC_BATCH_TUNED_DEF(8)
}  // namespace pimc
