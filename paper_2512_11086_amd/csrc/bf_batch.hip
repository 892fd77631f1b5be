// bf_batch.hip -- batched persistent decode + DAS and its hipGraph replay,
// plus the DAS tile autotuner.
#include "bf_plan.h"

namespace bf {
struct Batch {
};
}  // namespace bf

using namespace bf;

bf_plan_s::~bf_plan_s()
{
    magic = 0;
    delete batch;
    for (Frame *f : frames) delete f;
}

int64_t bf_plan_s::workspace_bytes() const
{
    int64_t b = 0;
    for (const Frame *f : frames) b += f->total_bytes;
    return b;
}

extern "C" {

int bf_batch_run(bf_plan plan, const int16_t *const *rf, float *const *out, void *stream)
{
    (void)plan; (void)rf; (void)out; (void)stream;
    return fail(BF_ERR_UNSUPPORTED, "batched path not built yet");
}

int bf_graph_launch(bf_plan plan, const int16_t *const *rf, float *const *out, void *stream)
{
    (void)plan; (void)rf; (void)out; (void)stream;
    return fail(BF_ERR_UNSUPPORTED, "batched path not built yet");
}

int bf_autotune(bf_plan plan, const char *cache_path)
{
    (void)plan; (void)cache_path;
    return fail(BF_ERR_UNSUPPORTED, "autotuner not built yet");
}

}  // extern "C"
