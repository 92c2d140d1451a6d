// kernels_csr_td.hip -- the CSR-form SpMV kernels for time-dependent Liouvillians.
//
// Same kernels as kernels_csr.hip (csr_kernels.h), instantiated with TD = true: every stored entry
// of the summed Liouvillian L(t) = L_0 + sum_k w_k(t) L_k carries its term number in the high bits
// of its column index, and the row sum weights it with the term's coefficient at the time of the
// evaluation (arXiv:2504.21440, Sec. 2, QobjEvo; Sec. 3.4).  The coefficient rows are written by
// the control and reset kernels, or by the stage-2 kernel that folds the control in.  A separate translation unit so the two kernel families compile
// in parallel.
#include "csr_kernels.h"

namespace qt {

void csr_td_spmv(const CsrLaunch &L, const CsrArgs &a, int first, int last)
{
    launch_spmv_range<true>(L, a, first, last);
}

bool csr_td_stage2_ctl(const CsrLaunch &L, const CsrArgs &a, const CsrCtl *rd, CsrCtl *wr)
{
    return launch_stage2_ctl<true>(L, a, rd, wr);
}

}  // namespace qt
