// Instantiations and launcher of the single-system hop for FP64 spinors and links (kernel template
// in wd_hop.hpp): the reliable updates, b_prec, eq. eo3, BiCGstab-M and wd_apply.
#include "wd_hop.hpp"

namespace wd {

hipError_t launch_hop64(bool dag, int lf, int red, const HopJob* jobs, int njobs, long nblocks, SysState* sys,
                        int gated, hipStream_t s, int* exec, int stage, int tg, int ntl, hipEvent_t ev0,
                        hipEvent_t ev1)
{
    const int sf = SF64;
    if (stage < 0) stage = hop_stage64_default();
    const int stage64 = stage;
    HOP_REDS(SF64, L64_18, false)
    HOP_REDS(SF64, L64_12, false)
    HOP_DAG_64(L64_18)
    HOP_DAG_64(L64_12)
    return hipErrorInvalidValue;
}

} // namespace wd
