// placeholder: serving queue entry points (implemented next)
#include "../../include/cayleygrowth.h"

extern "C" {
cg_queue_t *cg_queue_create(const cg_queue_opts_t *opts) { (void)opts; return nullptr; }
int cg_queue_submit(cg_queue_t *q, const cg_job_t *job, cg_result_t *res_slot, uint64_t *ticket) {
    (void)q; (void)job; (void)res_slot; (void)ticket; return CG_E_UNSUPPORTED;
}
int cg_queue_poll(cg_queue_t *q, uint64_t ticket) { (void)q; (void)ticket; return CG_E_UNSUPPORTED; }
int cg_queue_wait(cg_queue_t *q, uint64_t ticket, int64_t timeout_us) {
    (void)q; (void)ticket; (void)timeout_us; return CG_E_UNSUPPORTED;
}
int cg_queue_cancel(cg_queue_t *q, uint64_t ticket) { (void)q; (void)ticket; return CG_E_UNSUPPORTED; }
void cg_queue_destroy(cg_queue_t *q) { (void)q; }
}
