#include "problem.hpp"
using dlh::set_error;
extern "C" dl_status dl_batch_solve(dl_problem* const*, int32_t, const dl_solve_opts*, double* const*, dl_solve_result*, void*)
{ set_error("dl_batch_solve: not built yet"); return DL_ERR_UNSUPPORTED; }
extern "C" dl_status dl_server_create(size_t, int32_t, dl_server**) { set_error("not built yet"); return DL_ERR_UNSUPPORTED; }
extern "C" dl_status dl_server_submit(dl_server*, const dl_problem_desc*, const dl_problem_opts*, const dl_solve_opts*, uint64_t*) { set_error("not built yet"); return DL_ERR_UNSUPPORTED; }
extern "C" dl_status dl_server_poll(dl_server*, uint64_t, int32_t*, dl_solve_result*, double*) { set_error("not built yet"); return DL_ERR_UNSUPPORTED; }
extern "C" dl_status dl_server_times(dl_server*, uint64_t, double*, double*, double*) { set_error("not built yet"); return DL_ERR_UNSUPPORTED; }
extern "C" dl_status dl_server_destroy(dl_server*) { return DL_OK; }
