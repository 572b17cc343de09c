// Host-only C interface to the server's scheduler (serve_core.h), so that its
// allocator, residency and admission policy can be exercised without a GPU:
// the CPU tests drive it with a simulated device (requests with durations).
#include <cstdint>
#include <cstring>

#include "serve_core.h"

using gpspca::serve::Admission;
using gpspca::serve::Arena;
using gpspca::serve::Scheduler;
using gpspca::serve::Waiting;

extern "C" {

void* sched_create(size_t arena_bytes, int max_bypass) {
    return new Scheduler(arena_bytes, max_bypass);
}
void sched_destroy(void* s) { delete static_cast<Scheduler*>(s); }
void sched_add_matrix(void* s, uint64_t id, size_t bytes) {
    static_cast<Scheduler*>(s)->add_matrix(id, bytes);
}
int sched_remove_matrix(void* s, uint64_t id) {
    return static_cast<Scheduler*>(s)->remove_matrix(id) ? 1 : 0;
}
int sched_fits_alone(void* s, uint64_t matrix, size_t ws) {
    return static_cast<Scheduler*>(s)->fits_alone(matrix, ws) ? 1 : 0;
}
void sched_enqueue(void* s, uint64_t req, uint64_t matrix, size_t ws) {
    Waiting w;
    w.req = req;
    w.matrix = matrix;
    w.ws_bytes = ws;
    static_cast<Scheduler*>(s)->enqueue(w);
}
// Returns 1 and fills the outputs when a request was admitted.  `evicted`
// holds up to `cap` matrix ids; *n_evicted is the full count.
int sched_admit(void* s, uint64_t* req, uint64_t* matrix, uint64_t* ws_off, uint64_t* m_off,
                int* upload, uint64_t* evicted, int cap, int* n_evicted) {
    Admission a;
    const bool ok = static_cast<Scheduler*>(s)->admit(&a);
    *n_evicted = (int)a.evicted.size();
    for (int i = 0; i < (int)a.evicted.size() && i < cap; ++i) evicted[i] = a.evicted[i];
    if (!ok) return 0;
    *req = a.req;
    *matrix = a.matrix;
    *ws_off = a.ws_offset;
    *m_off = a.matrix_offset;
    *upload = a.upload ? 1 : 0;
    return 1;
}
void sched_finish(void* s, uint64_t matrix, uint64_t ws_off) {
    static_cast<Scheduler*>(s)->finish(matrix, (size_t)ws_off);
}
size_t sched_waiting(void* s) { return static_cast<Scheduler*>(s)->waiting(); }
size_t sched_free_bytes(void* s) { return static_cast<Scheduler*>(s)->arena().free_bytes(); }
size_t sched_arena_bytes(void* s) { return static_cast<Scheduler*>(s)->arena().size(); }
size_t sched_resident_bytes(void* s) { return static_cast<Scheduler*>(s)->resident_bytes(); }
uint64_t sched_evictions(void* s) { return static_cast<Scheduler*>(s)->evictions(); }
// Resident state of a matrix: -1 unknown, else resident flag | refs << 1.
int64_t sched_matrix_state(void* s, uint64_t id) {
    const auto* e = static_cast<Scheduler*>(s)->matrix(id);
    if (!e) return -1;
    return (e->resident ? 1 : 0) | ((int64_t)e->refs << 1);
}
// Blocks in use: writes up to cap (offset, length) pairs, returns the count.
int sched_used_blocks(void* s, uint64_t* out, int cap) {
    const auto v = static_cast<Scheduler*>(s)->arena().used_list();
    for (int i = 0; i < (int)v.size() && i < cap; ++i) {
        out[2 * i] = v[i].first;
        out[2 * i + 1] = v[i].second;
    }
    return (int)v.size();
}

// Bare allocator, for allocator property tests.
void* arena_create(size_t bytes) { return new Arena(bytes); }
void arena_destroy(void* a) { delete static_cast<Arena*>(a); }
uint64_t arena_alloc(void* a, size_t bytes) { return static_cast<Arena*>(a)->alloc(bytes); }
int arena_release(void* a, uint64_t off) { return static_cast<Arena*>(a)->release(off) ? 1 : 0; }
size_t arena_free_bytes(void* a) { return static_cast<Arena*>(a)->free_bytes(); }
size_t arena_largest_free(void* a) { return static_cast<Arena*>(a)->largest_free(); }

}  // extern "C"
