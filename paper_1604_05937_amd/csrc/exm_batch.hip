// Batched assembly (placeholder until the persistent kernel lands).
#include "exm_internal.hpp"

using namespace exm;

extern "C" {

int32_t exm_batch_create(int32_t, const exm_batch_item*, const exm_loop_opts*, void*, exm_batch** out)
{
    clear_error();
    if (out) *out = nullptr;
    return fail(EXM_EUNSUPPORTED, "batched assembly is not built yet");
}

int32_t exm_batch_launch(exm_batch*, void*)
{
    clear_error();
    return fail(EXM_EUNSUPPORTED, "batched assembly is not built yet");
}

int32_t exm_batch_info(const exm_batch*, int64_t*, int32_t*)
{
    clear_error();
    return fail(EXM_EUNSUPPORTED, "batched assembly is not built yet");
}

void exm_batch_destroy(exm_batch*) {}

}  // extern "C"
