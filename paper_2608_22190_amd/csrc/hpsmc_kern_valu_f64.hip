// Vector-unit round kernels, FP64 sampling precision.
#include "hpsmc_round.h"

namespace hpsmc {

hipError_t set_rec_tables_valu_f64() { return upload_recurrence_tables(); }

hipError_t launch_adv_valu_f64(const RoundArgs &a, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    return adv_d<double>(a, ns, grid, block, lds, s);
}

}  // namespace hpsmc
