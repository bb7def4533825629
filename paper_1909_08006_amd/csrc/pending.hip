// Entry points whose implementation files are not built yet.
#include "runtime.h"
using namespace ley;
extern "C" int leyenda_sort_runs(const void *, uint64_t, uint64_t, void *, uint64_t *, uint64_t, uint64_t *, void *) {
    return fail(LEYENDA_EINTERNAL, "leyenda_sort_runs: not built");
}
extern "C" int leyenda_merge(const void *, const uint64_t *, uint64_t, void *, uint64_t, void *) {
    return fail(LEYENDA_EINTERNAL, "leyenda_merge: not built");
}
extern "C" int leyenda_plan_runs(uint64_t, uint64_t, uint64_t *, uint64_t *) {
    return fail(LEYENDA_EINTERNAL, "leyenda_plan_runs: not built");
}
extern "C" int leyenda_sort_batch(const leyenda_segment *, uint64_t, void *) {
    return fail(LEYENDA_EINTERNAL, "leyenda_sort_batch: not built");
}
