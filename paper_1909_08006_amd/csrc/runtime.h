// Host-side helpers shared by the runtime translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdarg.h>

#include "../../include/leyenda.h"
#include "common.h"

namespace ley {

int fail(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
leyenda_params current_params();
Tune tune_of(const leyenda_params &p);
int device_cus();
int get_workspace(hipStream_t stream, size_t bytes, void **out);
int remember_layout(hipStream_t stream, const Layout &L);
// Pooled scratch slot `which` (0 or 1) of at least `bytes` for work on
// `stream`, kept between calls like the workspace (freed by
// leyenda_release_workspaces); a larger request replaces it after the stream drains.
int get_aux(hipStream_t stream, int which, size_t bytes, void **out);
void pool_forget(hipStream_t stream);
bool overlaps(const void *a, uint64_t abytes, const void *b, uint64_t bbytes);
int check_records(const void *in, const void *out, uint64_t n, const char *who);
// key_bytes (1..10): the key is that many leading bytes (10: the whole prefix).
// ties (n bytes, optional): ties[g] = 1 if output record g has the same key
// bytes 0..9 as output record g - 1, written by the record gather.
int sort_device(const void *records_dev, uint64_t n, void *out_dev, hipStream_t stream, const Tune &t,
                uint32_t key_bytes = kKeyBytes, uint8_t *ties = nullptr);
// Key bytes past key_bytes (1..10) cleared in the tuples a sort on w extracts.
void apply_key_mask(Work &w, uint32_t key_bytes);
// ORs the device-side guard word of the last sort of n records run on the
// workspace `ws` into *acc (device memory), in stream order on s.
hipError_t launch_guard_or(const void *ws, uint64_t n, const Tune &t, uint32_t *acc, hipStream_t s);
// The same for the last sort on `stream`'s pooled workspace (no-op if none ran).
int guard_or_pooled(hipStream_t stream, uint32_t *acc);
// Input record index per output position of the last sort of n records on
// `stream`'s pooled workspace (valid until the next sort there); null when no
// such sort ran or its indices name record-pool slots.
const uint32_t *pooled_sort_idx(hipStream_t stream, uint64_t n);
// Sorts n (key, index) tuples already written to buffer 0 (H[0], L[0]) of a
// workspace of plan_layout(n, 1, t).total bytes; the indices in key order end
// up in the workspace's idx array.  One output part, on stream s.
int sort_tuples_ws(uint64_t n, hipStream_t s, const Tune &t, void *ws);
// Same sort with a caller-provided workspace of plan_layout(n, 1, t).total bytes.
// bare: no phase-timing events and no side stream (one output part only).
// first_pass: kFirstSplit, or the first pass the workspace was laid out for
// (first_pass_for's choice for this n).
int sort_device_ws(const void *records_dev, uint64_t n, void *out_dev, hipStream_t stream, const Tune &t, void *ws,
                   uint32_t key_bytes = kKeyBytes, uint8_t *ties = nullptr, bool bare = false,
                   uint32_t first_pass = kFirstSplit);
uint32_t first_pass_for(uint64_t n, const Tune &t, bool ties);

// external.hip: the device arenas and bounce buffers the external calls keep
// between calls
bool external_holds_any();
void external_release_all();

// batch.hip
int batch_sort(const leyenda_segment *segs, uint64_t count, hipStream_t s);
// split: two-part launch sequence for the serving loop (see batch.hip); after
// a batch's first part completes, batch_continue_if_needed replays the second
// part when it is needed (returns 1), else returns 0 (negative: error).
int batch_reserve(hipStream_t s, uint64_t n, uint32_t r, size_t *bytes, bool split = false);
bool batch_is_split(hipStream_t s);
int batch_continue_if_needed(hipStream_t s);
uint64_t batch_bytes(uint64_t n, uint32_t r);
void batch_forget(hipStream_t s);
bool batch_holds_any();
void batch_release_all();

}  // namespace ley
