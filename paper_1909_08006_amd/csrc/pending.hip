// Entry points whose implementation files are not built yet.
#include "runtime.h"
using namespace ley;
extern "C" int leyenda_sort_batch(const leyenda_segment *, uint64_t, void *) {
    return fail(LEYENDA_EINTERNAL, "leyenda_sort_batch: not built");
}
