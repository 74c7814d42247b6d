// Test harness: the serving loop's host-only scheduler (the library's own
// sched.h, compiled with g++) behind a C interface, driven by the CPU tests
// with a simulated executor in place of the GPU.
#include "../paper_1902_03070_amd/csrc/sched.h"

extern "C" {

void* sh_new(int64_t budget, int max_active) {
    auto* s = new tsvd::Scheduler();
    s->configure(budget, max_active);
    return s;
}
void sh_free(void* s) { delete (tsvd::Scheduler*)s; }
int64_t sh_submit(void* s, int64_t footprint, double t, double deadline) {
    return ((tsvd::Scheduler*)s)->submit(footprint, t, deadline);
}
// Admits at time t; writes up to cap admitted ids; returns how many.
int sh_admit(void* s, double t, int64_t* ids, int cap) {
    auto v = ((tsvd::Scheduler*)s)->admit(t);
    int n = 0;
    for (int64_t id : v)
        if (n < cap) ids[n++] = id;
    return n;
}
void sh_expire(void* s, double t) { ((tsvd::Scheduler*)s)->expire(t); }
int sh_take_stopped(void* s, double t, int64_t* ids, int* codes, int cap) {
    auto v = ((tsvd::Scheduler*)s)->take_stopped(t);
    int n = 0;
    for (auto& e : v)
        if (n < cap) {
            ids[n] = e.first;
            codes[n] = e.second;
            ++n;
        }
    return n;
}
int sh_cancel(void* s, int64_t id, double t) { return ((tsvd::Scheduler*)s)->cancel(id, t); }
void sh_finish(void* s, int64_t id, int status) { ((tsvd::Scheduler*)s)->finish(id, status); }
int sh_state(void* s, int64_t id) { return ((tsvd::Scheduler*)s)->state(id); }
int sh_status(void* s, int64_t id) { return ((tsvd::Scheduler*)s)->status(id); }
void sh_forget(void* s, int64_t id) { ((tsvd::Scheduler*)s)->forget(id); }
int64_t sh_held(void* s) { return ((tsvd::Scheduler*)s)->held(); }
int64_t sh_peak(void* s) { return ((tsvd::Scheduler*)s)->peak(); }
int sh_active(void* s) { return ((tsvd::Scheduler*)s)->active(); }
int64_t sh_queued(void* s) { return ((tsvd::Scheduler*)s)->queued(); }
int64_t sh_completed(void* s) { return ((tsvd::Scheduler*)s)->completed(); }
}
