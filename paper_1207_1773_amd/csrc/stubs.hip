// Temporary placeholders for stages not yet written.
#include "hgv_internal.h"
namespace hgv {
struct StageMissing {};
void he2hb_run(hgv_ctx_s *, int, int, double2 *, int, double2 *, Arena &ar) { if (!ar.measuring()) throw HipFail{hipErrorNotSupported}; }
void hb2st_run(hgv_ctx_s *, int, int, const double2 *, int, double *, double *, double2 *, double2 *, Arena &ar) { if (!ar.measuring()) throw HipFail{hipErrorNotSupported}; }
size_t v2_elems(int n, int nb) { return (size_t)n * n + nb; }
size_t v2_taus(int n, int nb) { return (size_t)n * n / nb + 1; }
void stedc_run(hgv_ctx_s *, int, const double *, const double *, int, int, double *, double *, int, Arena &ar, int *) { if (!ar.measuring()) throw HipFail{hipErrorNotSupported}; }
void unmtr_q2_run(hgv_ctx_s *, int, int, int, const double2 *, const double2 *, double2 *, int, Arena &ar) { if (!ar.measuring()) throw HipFail{hipErrorNotSupported}; }
void unmtr_q1_run(hgv_ctx_s *, int, int, int, const double2 *, int, const double2 *, double2 *, int, Arena &ar) { if (!ar.measuring()) throw HipFail{hipErrorNotSupported}; }
}
