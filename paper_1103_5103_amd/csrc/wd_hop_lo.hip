// Instantiations and launcher of the single-system hop for FP32 / FP16 spinors (kernel template in
// wd_hop.hpp); FP64 launches go to launch_hop64 (wd_hop64.hip).
#include "wd_hop.hpp"

namespace wd {

hipError_t launch_hop64(bool dag, int lf, int red, const HopJob* jobs, int njobs, long nblocks, SysState* sys,
                        int gated, hipStream_t s, int* exec, int stage, int tg, int ntl, hipEvent_t ev0,
                        hipEvent_t ev1);

hipError_t launch_hop(int sf, int lf, bool dag, int red, int fin, const HopJob* jobs, int njobs, long nblocks,
                      SysState* sys, int gated, hipStream_t s, int* exec, int stage, int tg, int ntl, hipEvent_t ev0,
                      hipEvent_t ev1)
{
    if (tg && dag) return hipErrorInvalidValue;  // the adjoint hop runs on the caller's links only
    if (nblocks <= 0) return hipSuccess;
    if (sf == SF64) return launch_hop64(dag, lf, red, jobs, njobs, nblocks, sys, gated, s, exec, stage, tg, ntl, ev0, ev1);
    if (stage < 0) stage = hop_stage_default();
    const int stage64 = stage;
    HOP_REDS(SF32, L32_12, false)
    HOP_REDS(SF32, L16_12, false)
    HOP_REDS(SF32, LB16_12, false)
    HOP_REDS(SF16, L32_12, false)
    HOP_REDS(SF16, L16_12, false)
    HOP_REDS(SF16, LB16_12, false)
    HOP_REDS(SF32, L16_8, false)
    HOP_REDS(SF16, L16_8, false)
    HOP_DAG_LO(SF32, L32_12)
    HOP_DAG_LO(SF32, L16_12)
    HOP_DAG_LO(SF32, LB16_12)
    HOP_DAG_LO(SF16, L32_12)
    HOP_DAG_LO(SF16, L16_12)
    HOP_DAG_LO(SF16, LB16_12)
    HOP_DAG_LO(SF32, L16_8)
    HOP_DAG_LO(SF16, L16_8)
    (void)stage64;
    (void)fin;
    return hipErrorInvalidValue;
}

} // namespace wd
