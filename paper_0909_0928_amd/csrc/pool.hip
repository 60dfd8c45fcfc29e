// Request pool: registrations of any size submitted by the caller are run on
// a fixed set of slots (a handle with its own stream each), admitted in
// arrival order while a slot is free and the workspace the slots hold stays
// within a byte budget, so requests that arrive while others run overlap with
// them on the device.  With a batch limit above 1, the request at the head of
// the queue is admitted together with the queued requests after it that can
// run in lockstep with it (the same levels, iterations, sigma, radius,
// storage, units and image pre-smoothing, and in mm the same spacing), up to that limit, as one lockstep batch on one slot.  The pool is
// driven by the caller's calls (no thread of its own): every call first
// collects finished registrations, without blocking, and admits queued ones.
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
    hipEvent_t done = nullptr;          // recorded after the registration's work
    int count = 0;                      // registrations running (0: free)
    int64_t tickets[DIR_MAX_BATCH] = {};
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
    int max_batch = 1;    // registrations one slot may run in lockstep
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
        if (!s.count) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        dir_stats st[DIR_MAX_BATCH];
        int32_t status[DIR_MAX_BATCH];
        memset(st, 0, sizeof st);
        for (int r = 0; r < s.count; ++r) {
            st[r].struct_size = sizeof(dir_stats);
            status[r] = DIR_EDEVICE;
        }
        const int rc = dir::collect_each(s.h, st, status);
        for (int r = 0; r < s.count; ++r) {
            Result res;
            res.stats = st[r];
            res.status = (q != hipSuccess || (rc != DIR_OK && rc != DIR_ENUMERIC)) ? DIR_EDEVICE : status[r];
            p->results[s.tickets[r]] = res;
        }
        s.count = 0;
    }
    return DIR_OK;
}

// Whether request b can run in lockstep with request a.
bool lockstep_with(const Request &a, const Request &b)
{
    const dir_params &x = a.params, &y = b.params;
    if (x.levels != y.levels || x.sigma != y.sigma || x.radius != y.radius || x.storage != y.storage) return false;
    if (x.units != y.units || x.image_sigma != y.image_sigma) return false;
    if (x.units == DIR_UNITS_MM && memcmp(a.spacing, b.spacing, sizeof a.spacing) != 0) return false;
    for (int l = 0; l < x.levels; ++l)
        if (x.iters[l] != y.iters[l]) return false;
    return true;
}

// The head request and the queued ones that can join it, in queue order.
struct Group {
    int count = 0;
    int idx[DIR_MAX_BATCH];  // queue positions
    int32_t dims[3 * DIR_MAX_BATCH];
    dir_params params[DIR_MAX_BATCH];
};

Group head_group(const dir_pool *p)
{
    Group g;
    const Request &head = p->queue.front();
    for (int i = 0; i < (int)p->queue.size() && g.count < p->max_batch; ++i) {
        const Request &q = p->queue[i];
        if (i > 0 && (!lockstep_with(head, q) || q.has_spacing != head.has_spacing)) continue;
        g.idx[g.count] = i;
        g.dims[3 * g.count] = q.nx;
        g.dims[3 * g.count + 1] = q.ny;
        g.dims[3 * g.count + 2] = q.nz;
        g.params[g.count] = q.params;
        ++g.count;
    }
    return g;
}

// Workspace slot s holds after running group g.
uint64_t bytes_after(const Slot &s, const Group &g)
{
    return g.count == 1 ? dir::workspace_after(s.h, g.dims[0], g.dims[1], g.dims[2], &g.params[0])
                        : dir::workspace_after_batch(s.h, g.count, g.dims, g.params);
}

// Enqueue group g on slot s; the requests' results on failure.
void start(dir_pool *p, Slot &s, const Group &g)
{
    const float *S[DIR_MAX_BATCH], *M[DIR_MAX_BATCH];
    float *out[DIR_MAX_BATCH];
    double spacing[3 * DIR_MAX_BATCH];
    int64_t tickets[DIR_MAX_BATCH];
    for (int r = 0; r < g.count; ++r) {
        const Request &q = p->queue[g.idx[r]];
        S[r] = q.S;
        M[r] = q.M;
        out[r] = q.out;
        tickets[r] = q.ticket;
        for (int k = 0; k < 3; ++k) spacing[3 * r + k] = q.spacing[k];
    }
    const bool has_spacing = p->queue[g.idx[0]].has_spacing;
    int32_t rc;
    if (g.count == 1)
        rc = dir_register_async(s.h, S[0], M[0], g.dims[0], g.dims[1], g.dims[2], has_spacing ? spacing : nullptr,
                                &g.params[0], out[0]);
    else
        rc = dir_register_batch_async(s.h, g.count, S, M, g.dims, has_spacing ? spacing : nullptr, g.params, out);
    if (rc == DIR_OK && hipEventRecord(s.done, s.stream) != hipSuccess) {
        dir::collect_each(s.h, nullptr, nullptr);
        rc = DIR_EDEVICE;
    }
    if (rc == DIR_OK) {
        s.count = g.count;
        for (int r = 0; r < g.count; ++r) s.tickets[r] = tickets[r];
    } else {
        for (int r = 0; r < g.count; ++r) p->results[tickets[r]] = Result{rc, {}};
    }
    for (int r = g.count - 1; r >= 0; --r) p->queue.erase(p->queue.begin() + g.idx[r]);  // positions ascend
}

// Admit queued requests in order while the head (with as much of its group
// as fits) fits.
int32_t admit(dir_pool *p)
{
    while (!p->queue.empty()) {
        Group g = head_group(p);
        int chosen = -1;
        while (chosen < 0) {
            // the free slot whose workspace grows least
            int best = -1;
            uint64_t best_growth = 0;
            for (int i = 0; i < (int)p->slots.size(); ++i) {
                const Slot &s = p->slots[i];
                if (s.count) continue;
                const uint64_t gr = bytes_after(s, g) - dir::workspace_now(s.h);
                if (best < 0 || gr < best_growth) {
                    best = i;
                    best_growth = gr;
                }
            }
            if (best < 0) return DIR_OK;  // every slot busy
            Slot &s = p->slots[best];
            bool fits = !p->budget || held_bytes(p) + best_growth <= p->budget;
            if (!fits) {
                // give back the workspace of the other free slots, then this one's
                for (Slot &o : p->slots)
                    if (!o.count && &o != &s) dir::workspace_release(o.h);
                fits = held_bytes(p) + (bytes_after(s, g) - dir::workspace_now(s.h)) <= p->budget;
                if (!fits) {
                    dir::workspace_release(s.h);
                    fits = held_bytes(p) + bytes_after(s, g) <= p->budget;
                }
            }
            if (fits) chosen = best;
            else if (g.count > 1) --g.count;  // a smaller group (down to the head alone, which fits an idle pool)
            else return DIR_OK;               // wait for a running registration
        }
        start(p, p->slots[chosen], g);
        const uint64_t held = held_bytes(p);
        if (held > p->peak_bytes) p->peak_bytes = held;
        int32_t running = 0;
        for (const Slot &o : p->slots) running += o.count;
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
        for (int r = 0; r < p->slots[i].count; ++r)
            if (p->slots[i].tickets[r] == t) return i;
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
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
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
    (void)hipSetDevice(p->device);
    for (Slot &s : p->slots) {
        if (s.count) dir::collect_each(s.h, nullptr, nullptr);
        dir_destroy(s.h);
        (void)hipEventDestroy(s.done);
        (void)hipStreamDestroy(s.stream);
    }
    delete p;
    return DIR_OK;
}

int32_t dir_pool_set_max_batch(dir_pool *p, int32_t max_batch)
{
    if (!p || max_batch < 1 || max_batch > DIR_MAX_BATCH) return DIR_EINVAL;
    p->max_batch = max_batch;
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
                if (p->slots[k].count) i = k;
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
