// placeholder batch entry points
#include "vegas.h"
extern "C" {
vegas_status vegas_batch_workspace_size(const vegas_desc*, const int64_t*, int32_t, size_t*) { return VEGAS_EUNSUPPORTED; }
vegas_status vegas_batch_plan(vegas_batch** out, const vegas_desc*, const int64_t*, int32_t, void*, size_t, int32_t, int32_t, vegas_stream_t) { if (out) *out = nullptr; return VEGAS_EUNSUPPORTED; }
vegas_status vegas_batch_run(vegas_batch*, vegas_stream_t) { return VEGAS_EUNSUPPORTED; }
vegas_status vegas_batch_results(vegas_batch*, vegas_result_t*, vegas_stream_t) { return VEGAS_EUNSUPPORTED; }
vegas_status vegas_batch_get_edges(vegas_batch*, int32_t, double*, vegas_stream_t) { return VEGAS_EUNSUPPORTED; }
vegas_status vegas_batch_destroy(vegas_batch*) { return VEGAS_OK; }
}
