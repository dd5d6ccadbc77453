// ftgemm_lp_ilp.hip -- the low-precision kernels that the build compiles with
// the compiler's iterative ILP scheduling strategy (see launch_own_unit in
// ftgemm_lp.hip for which, and why): the same source, included with
// FTG_LP_OWN_UNIT defined, so that this translation unit holds only those
// kernels and their launch function.
#define FTG_LP_OWN_UNIT 1
#include "ftgemm_lp.hip"
