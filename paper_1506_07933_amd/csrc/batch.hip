// batch.hip -- batched uneven-size executor (placeholder).
#include "plan.hpp"

namespace mifft {
int batch_create(mifft_batch*, int, const int*, int, int, unsigned)
{
    return set_error(MIFFT_ERR_UNSUPPORTED, "batched execution is not built yet");
}
int batch_execute(mifft_batch, void* const*, void* const*, void*, bool)
{
    return set_error(MIFFT_ERR_BADPLAN, "batched execution is not built yet");
}
int batch_destroy(mifft_batch b) { return b ? set_error(MIFFT_ERR_BADPLAN, "not a batch") : MIFFT_OK; }
} // namespace mifft
