// Split-precision contraction (BF16 / INT8 digit products on matrix cores, FP64 recombination).
#include "context.hpp"

namespace flapw {

flapw_status split_contraction(flapw_handle h, long long kp2, const std::vector<ProblemDev> &probs,
                               const std::vector<TileDev> &tiles, flapw_prec prec, int slices, hipStream_t s)
{
    (void)kp2; (void)probs; (void)tiles; (void)prec; (void)slices; (void)s;
    return fail(h, FLAPW_ERR_UNSUPPORTED, "split precision is not built yet");
}

void split_release(flapw_handle h)
{
    h->digits.release();
    h->sdesc.release();
}

long long split_bytes(flapw_handle h) { return (long long)(h->digits.n + h->sdesc.n); }

}  // namespace flapw
