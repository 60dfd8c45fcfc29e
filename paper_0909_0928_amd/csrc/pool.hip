// Request pool: registrations of any size submitted by the caller are run on
// a fixed set of slots (a handle with its own stream each), admitted in
// arrival order while a slot is free and the workspace the slots hold stays
// within a byte budget, so requests that arrive while others run overlap with
// them on the device.  The pool is driven by the caller's calls (no thread of
// its own): every call first collects finished registrations, without
// blocking, and admits queued ones.
#include <hip/hip_runtime.h>
#include <string.h>

#include <deque>
#include <map>
#include <new>
#include <vector>

#include "demons.h"
#include "dir_internal.h"

namespace {

struct Slot {
    dir_handle *h = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;  // recorded after the registration's work
    int64_t ticket = 0;         // 0: free
};

struct Request {
    int64_t ticket;
    const float *S, *M;
    float *out;
    int32_t nx, ny, nz;
    dir_params params;
    bool has_spacing;
    double spacing[3];
};

struct Result {
    int32_t status;
    dir_stats stats;
};

}  // namespace

struct dir_pool {
    int device = 0;
    uint64_t budget = 0;  // 0: no limit
    std::vector<Slot> slots;
    std::deque<Request> queue;
    std::map<int64_t, Result> results;
    int64_t next_ticket = 1;
    uint64_t peak_bytes = 0;
    int32_t peak_running = 0;
};

namespace {

uint64_t held_bytes(const dir_pool *p)
{
    uint64_t b = 0;
    for (const Slot &s : p->slots) b += dir::workspace_now(s.h);
    return b;
}

// Move finished registrations from their slots to the results.
int32_t collect(dir_pool *p)
{
    for (Slot &s : p->slots) {
        if (!s.ticket) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        Result r;
        memset(&r.stats, 0, sizeof r.stats);
        r.stats.struct_size = sizeof(dir_stats);
        r.status = q == hipSuccess ? dir_wait(s.h, &r.stats) : DIR_EDEVICE;
        if (q != hipSuccess) dir_wait(s.h, nullptr);
        p->results[s.ticket] = r;
        s.ticket = 0;
    }
    return DIR_OK;
}

// Admit queued requests in order while one fits.
int32_t admit(dir_pool *p)
{
    while (!p->queue.empty()) {
        const Request &q = p->queue.front();
        // the free slot whose workspace grows least
        int best = -1;
        uint64_t best_growth = 0;
        for (int i = 0; i < (int)p->slots.size(); ++i) {
            const Slot &s = p->slots[i];
            if (s.ticket) continue;
            const uint64_t g = dir::workspace_after(s.h, q.nx, q.ny, q.nz, &q.params) - dir::workspace_now(s.h);
            if (best < 0 || g < best_growth) {
                best = i;
                best_growth = g;
            }
        }
        if (best < 0) return DIR_OK;  // every slot busy
        Slot &s = p->slots[best];
        if (p->budget) {
            uint64_t after = held_bytes(p) + best_growth;
            if (after > p->budget) {
                // give back the workspace of the other free slots, then this one's
                for (Slot &o : p->slots)
                    if (!o.ticket && &o != &s) dir::workspace_release(o.h);
                after = held_bytes(p) + (dir::workspace_after(s.h, q.nx, q.ny, q.nz, &q.params) -
                                         dir::workspace_now(s.h));
                if (after > p->budget) {
                    dir::workspace_release(s.h);
                    after = held_bytes(p) + dir::workspace_after(s.h, q.nx, q.ny, q.nz, &q.params);
                }
                if (after > p->budget) return DIR_OK;  // wait for a running registration
            }
        }
        const int32_t rc = dir_register_async(s.h, q.S, q.M, q.nx, q.ny, q.nz, q.has_spacing ? q.spacing : nullptr,
                                              &q.params, q.out);
        if (rc == DIR_OK) {
            const hipError_t e = hipEventRecord(s.done, s.stream);
            if (e != hipSuccess) {
                dir_wait(s.h, nullptr);
                p->results[q.ticket] = Result{DIR_EDEVICE, {}};
            } else {
                s.ticket = q.ticket;
            }
        } else {
            Result r{rc, {}};
            p->results[q.ticket] = r;
        }
        p->queue.pop_front();
        const uint64_t held = held_bytes(p);
        if (held > p->peak_bytes) p->peak_bytes = held;
        int32_t running = 0;
        for (const Slot &o : p->slots) running += o.ticket ? 1 : 0;
        if (running > p->peak_running) p->peak_running = running;
    }
    return DIR_OK;
}

int32_t progress(dir_pool *p)
{
    if (hipSetDevice(p->device) != hipSuccess) return DIR_EDEVICE;
    collect(p);
    return admit(p);
}

bool queued(const dir_pool *p, int64_t t)
{
    for (const Request &q : p->queue)
        if (q.ticket == t) return true;
    return false;
}

int running_slot(const dir_pool *p, int64_t t)
{
    for (int i = 0; i < (int)p->slots.size(); ++i)
        if (p->slots[i].ticket == t) return i;
    return -1;
}

int32_t take_result(dir_pool *p, int64_t t, dir_stats *stats)
{
    auto it = p->results.find(t);
    const int32_t status = it->second.status;
    if (stats) {
        double *hist = stats->history;
        const int32_t cap = stats->history_capacity;
        *stats = it->second.stats;
        stats->history = hist;  // histories are not kept by the pool
        stats->history_capacity = cap;
        stats->history_len = 0;
    }
    p->results.erase(it);
    return status;
}

}  // namespace

extern "C" {

int32_t dir_pool_create(dir_pool **out, int32_t device, int32_t slots, uint64_t max_bytes)
{
    if (!out || slots < 1 || slots > 64) return DIR_EINVAL;
    *out = nullptr;
    dir_pool *p = new (std::nothrow) dir_pool();
    if (!p) return DIR_ENOMEM;
    p->device = device;
    p->budget = max_bytes;
    if (hipSetDevice(device) != hipSuccess) {
        delete p;
        return DIR_EINVAL;
    }
    for (int i = 0; i < slots; ++i) {
        Slot s;
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            dir_create(&s.h, device, s.stream) != DIR_OK) {
            if (s.h) dir_destroy(s.h);
            if (s.done) hipEventDestroy(s.done);
            if (s.stream) hipStreamDestroy(s.stream);
            dir_pool_destroy(p);
            return DIR_EDEVICE;
        }
        p->slots.push_back(s);
    }
    *out = p;
    return DIR_OK;
}

int32_t dir_pool_destroy(dir_pool *p)
{
    if (!p) return DIR_OK;
    hipSetDevice(p->device);
    for (Slot &s : p->slots) {
        if (s.ticket) dir_wait(s.h, nullptr);
        dir_destroy(s.h);
        hipEventDestroy(s.done);
        hipStreamDestroy(s.stream);
    }
    delete p;
    return DIR_OK;
}

int32_t dir_pool_submit(dir_pool *p, const float *d_static, const float *d_moving, int32_t nx, int32_t ny,
                        int32_t nz, const double *spacing_mm, const dir_params *params, float *d_field_out,
                        int64_t *ticket)
{
    if (!p || !ticket || !d_static || !d_moving || !d_field_out) return DIR_EINVAL;
    uint64_t need = 0;
    const int32_t rc = dir_workspace_bytes(nx, ny, nz, params, &need);
    if (rc != DIR_OK) return rc;
    if (p->budget && need > p->budget) return DIR_ENOMEM;
    Request q;
    q.ticket = p->next_ticket++;
    q.S = d_static;
    q.M = d_moving;
    q.out = d_field_out;
    q.nx = nx;
    q.ny = ny;
    q.nz = nz;
    q.params = *params;
    q.has_spacing = spacing_mm != nullptr;
    for (int k = 0; k < 3; ++k) q.spacing[k] = spacing_mm ? spacing_mm[k] : 1.0;
    p->queue.push_back(q);
    *ticket = q.ticket;
    return progress(p);
}

int32_t dir_pool_progress(dir_pool *p)
{
    if (!p) return DIR_EINVAL;
    return progress(p);
}

int32_t dir_pool_poll(dir_pool *p, int64_t ticket, dir_stats *stats, int32_t *done)
{
    if (!p || !done) return DIR_EINVAL;
    if (stats && stats->struct_size != (int32_t)sizeof(dir_stats)) return DIR_EINVAL;
    const int32_t rc = progress(p);
    if (rc != DIR_OK) return rc;
    if (p->results.count(ticket)) {
        *done = 1;
        return take_result(p, ticket, stats);
    }
    *done = 0;
    return (queued(p, ticket) || running_slot(p, ticket) >= 0) ? DIR_OK : DIR_EINVAL;
}

int32_t dir_pool_wait(dir_pool *p, int64_t ticket, dir_stats *stats)
{
    if (!p) return DIR_EINVAL;
    if (stats && stats->struct_size != (int32_t)sizeof(dir_stats)) return DIR_EINVAL;
    for (;;) {
        const int32_t rc = progress(p);
        if (rc != DIR_OK) return rc;
        if (p->results.count(ticket)) return take_result(p, ticket, stats);
        int i = running_slot(p, ticket);
        if (i < 0 && !queued(p, ticket)) return DIR_EINVAL;
        if (i < 0) {  // queued: wait for the oldest running registration to free room
            for (int k = 0; k < (int)p->slots.size() && i < 0; ++k)
                if (p->slots[k].ticket) i = k;
            if (i < 0) return DIR_EDEVICE;  // nothing runs and it was not admitted: cannot happen
        }
        if (hipEventSynchronize(p->slots[i].done) != hipSuccess) return DIR_EDEVICE;
    }
}

int32_t dir_pool_stats(const dir_pool *p, uint64_t *held_bytes_now, uint64_t *peak_bytes, int32_t *peak_running,
                       int32_t *queued_now)
{
    if (!p) return DIR_EINVAL;
    if (held_bytes_now) *held_bytes_now = held_bytes(p);
    if (peak_bytes) *peak_bytes = p->peak_bytes;
    if (peak_running) *peak_running = p->peak_running;
    if (queued_now) *queued_now = (int32_t)p->queue.size();
    return DIR_OK;
}

}  // extern "C"
