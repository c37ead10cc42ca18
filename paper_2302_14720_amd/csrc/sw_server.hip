// sw_server.hip -- serving runtime: independent SW jobs (lattice side, beta,
// J, seed, number of sweeps) share one GPU.  Each job's buffers are carved
// from one device memory pool; jobs wait in a FIFO queue until their
// footprint fits, then join the active set, and every step advances all
// active jobs together through the batched kernels (one launch per kernel
// of a sweep for all jobs of a tile width).  A job's randomness depends only
// on its seed, its own sweep counter and the site, so its records and spins
// are bit for bit those of a plain sim run alone.  When a job reaches its
// sweep count it leaves the active set (its spins are resolved to +-1 and
// its records stay readable until it is released), and queued jobs are
// admitted into the freed memory.
#include <string.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "sw_host.h"

using swmi::Dev;
using swmi::fail;

namespace {

struct Job {
    int64_t id = 0;
    sw_config cfg{};
    Dev dev{};
    size_t off = 0, bytes = 0;
    int64_t target = 0, done = 0;
    int32_t state = SW_JOB_QUEUED;
    int32_t slot = -1;
};

// First-fit allocator over [0, size) with coalescing of freed ranges.
struct Pool {
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_;  // offset -> length

    void init(size_t n) {
        size = n;
        used = 0;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Launch groups: Ising and Potts jobs, each with 64-wide or 32-wide tiles,
// run different instantiations of the tile and resolve kernels.
constexpr int kGroups = 4;
int group_of(const Dev &d) { return (d.q ? 2 : 0) + (d.tw == 64 ? 0 : 1); }
void set_groups(swmi::BatchDev *bd) {
    for (int g = 0; g < kGroups; ++g) {
        bd[g].tw = (g & 1) ? 32u : 64u;
        bd[g].potts = g >= 2 ? 1u : 0u;
    }
}

}  // namespace

struct sw_server {
    void *pool_mem = nullptr;
    bool own_pool = false;
    Pool pool;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int32_t max_jobs = 0;
    Dev *d_devs = nullptr;      // [max_jobs] Dev of the job in each slot
    uint32_t *d_maps = nullptr;  // map entries of the current launch groups
    size_t maps_cap = 0;
    std::vector<int32_t> free_slots;
    std::unordered_map<int64_t, Job *> jobs;
    std::deque<Job *> queue;
    std::vector<Job *> active;
    int64_t next_id = 1;
    bool dirty = true;
    swmi::BatchDev bd[kGroups]{};  // active jobs by launch group (see group_of)
    uint64_t site_updates = 0;
};

namespace {

int srv_device(const sw_server *s) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != s->device) HIP_TRY(hipSetDevice(s->device));
    return SW_OK;
}

// Copies the maps of the launch groups into the device map buffer and
// points the BatchDevs at them.  The stream is idle when this runs.
int upload_maps(sw_server *s, swmi::BatchMaps *m, swmi::BatchDev *bd, int ngroups) {
    size_t need = 0;
    for (int i = 0; i < ngroups; ++i) need += m[i].words();
    if (need > s->maps_cap) {
        if (s->d_maps) (void)hipFree(s->d_maps);
        s->d_maps = nullptr;
        s->maps_cap = 0;
        const size_t cap = std::max<size_t>(need * 2, 4096);
        const hipError_t e = hipMalloc(&s->d_maps, cap * 4);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SW_ENOMEM, "hipMalloc of the server's work maps failed");
        }
        s->maps_cap = cap;
    }
    std::vector<uint32_t> host;
    host.reserve(need);
    for (int i = 0; i < ngroups; ++i) {
        bd[i].devs = s->d_devs;
        m[i].emit(host, s->d_maps, bd[i]);
    }
    if (!host.empty()) HIP_TRY(hipMemcpy(s->d_maps, host.data(), host.size() * 4, hipMemcpyHostToDevice));
    return SW_OK;
}

int rebuild_active(sw_server *s) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    swmi::BatchMaps m[kGroups];
    for (Job *j : s->active) m[group_of(j->dev)].add((uint32_t)j->slot, j->dev, true);
    set_groups(s->bd);
    const int rc = upload_maps(s, m, s->bd, kGroups);
    if (rc == SW_OK) s->dirty = false;
    return rc;
}

// Moves queued jobs (in order) into the active set while memory and slots
// allow; a job that does not fit waits, and so do the jobs behind it.
int admit(sw_server *s) {
    while (!s->queue.empty() && !s->free_slots.empty()) {
        Job *j = s->queue.front();
        size_t off = 0;
        if (!s->pool.alloc(j->bytes, &off)) break;
        const int32_t slot = s->free_slots.back();
        char *base = (char *)s->pool_mem + off;
        const Dev dev = swmi::make_dev(j->cfg, base, swmi::layout_of(j->cfg));
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess) e = hipMemsetAsync(base, 0, j->bytes, s->stream);
        if (e == hipSuccess) e = swmi::launch_init(dev, j->cfg.init == SW_INIT_COLD ? 1 : 0, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess) e = hipMemcpy(s->d_devs + slot, &dev, sizeof(Dev), hipMemcpyHostToDevice);
        if (e != hipSuccess) {  // the job stays queued; its memory and slot are returned
            s->pool.release(off, j->bytes);
            return swmi::hip_fail(e, "admitting a job");
        }
        s->queue.pop_front();
        s->free_slots.pop_back();
        j->off = off;
        j->slot = slot;
        j->dev = dev;
        j->state = SW_JOB_ACTIVE;
        s->active.push_back(j);
        s->dirty = true;
    }
    return SW_OK;
}

int find_job(sw_server *s, int64_t id, Job **out) {
    if (!s) return fail(SW_EINVAL, "server is NULL");
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(SW_ERANGE, "unknown job id " + std::to_string(id));
    *out = it->second;
    return SW_OK;
}

sw_config job_config(int32_t L, double beta, double J, uint64_t seed, int32_t q, int32_t init, int64_t sweeps) {
    sw_config c;
    sw_config_init(&c, L, beta, J, seed);
    c.q = q;
    c.init = init;
    c.ring = sweeps;
    return c;
}

int submit(sw_server *s, const sw_config &c, int64_t sweeps, int64_t *job_id) {
    int rc = swmi::validate(&c);
    if (rc != SW_OK) return rc;
    const size_t bytes = swmi::align_up(swmi::layout_of(c).total);
    if (bytes > s->pool.size)
        return fail(SW_ENOMEM, "job needs " + std::to_string(bytes) + " bytes, more than the whole pool");
    Job *j = new (std::nothrow) Job();
    if (!j) return fail(SW_ENOMEM, "host allocation failed");
    j->id = s->next_id++;
    j->cfg = c;
    j->bytes = bytes;
    j->target = sweeps;
    s->jobs[j->id] = j;
    s->queue.push_back(j);
    *job_id = j->id;
    return SW_OK;
}

}  // namespace

extern "C" {

size_t sw_server_job_bytes(int32_t L, int64_t sweeps) { return sw_server_job_bytes_potts(L, 0, sweeps); }

size_t sw_server_job_bytes_potts(int32_t L, int32_t q, int64_t sweeps) {
    if (sweeps < 1) return 0;
    const sw_config c = job_config(L, 0.0, 1.0, 0, q, SW_INIT_HOT, sweeps);
    if (swmi::validate(&c) != SW_OK) return 0;
    return swmi::align_up(swmi::layout_of(c).total);
}

int sw_server_create(void *pool, size_t pool_bytes, int32_t max_jobs, void *hip_stream, sw_server **out) {
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_jobs < 1 || max_jobs > swmi::kMaxReplicas)
        return fail(SW_EINVAL, "max_jobs must be in [1, " + std::to_string(swmi::kMaxReplicas) + "]");
    if (pool_bytes < swmi::kAlign) return fail(SW_EINVAL, "pool_bytes is too small");
    if (pool && ((uintptr_t)pool % swmi::kAlign) != 0) return fail(SW_EINVAL, "pool must be 256-byte aligned");
    sw_server *s = new (std::nothrow) sw_server();
    if (!s) return fail(SW_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return swmi::hip_fail(e, "hipGetDevice");
    }
    pool_bytes &= ~(swmi::kAlign - 1);
    if (pool) {
        s->pool_mem = pool;
    } else {
        e = hipMalloc(&s->pool_mem, pool_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return fail(SW_ENOMEM, "hipMalloc of the " + std::to_string(pool_bytes) + "-byte pool failed");
        }
        s->own_pool = true;
    }
    s->pool.init(pool_bytes);
    s->max_jobs = max_jobs;
    e = hipMalloc((void **)&s->d_devs, (size_t)max_jobs * sizeof(Dev));
    if (e == hipSuccess) {
        if (hip_stream) {
            s->stream = (hipStream_t)hip_stream;
        } else {
            e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
            s->own_stream = e == hipSuccess;
        }
    }
    if (e != hipSuccess) {
        const int rc = swmi::hip_fail(e, "creating the server");
        sw_server_destroy(s);
        return rc;
    }
    for (int32_t i = max_jobs - 1; i >= 0; --i) s->free_slots.push_back(i);
    *out = s;
    return SW_OK;
}

int sw_server_submit(sw_server *s, int32_t L, double beta, double J, uint64_t seed, int32_t init, int64_t sweeps,
                     int64_t *job_id) {
    if (!s || !job_id) return fail(SW_EINVAL, "server or job_id is NULL");
    if (sweeps < 1) return fail(SW_EINVAL, "sweeps must be >= 1");
    return submit(s, job_config(L, beta, J, seed, 0, init, sweeps), sweeps, job_id);
}

int sw_server_submit_potts(sw_server *s, int32_t L, double beta, double J, uint64_t seed, int32_t q, int32_t init,
                           int64_t sweeps, int64_t *job_id) {
    if (!s || !job_id) return fail(SW_EINVAL, "server or job_id is NULL");
    if (sweeps < 1) return fail(SW_EINVAL, "sweeps must be >= 1");
    if (q < 2 || q > swmi::kMaxQ) return fail(SW_EINVAL, "Potts q must be in [2, 8]");
    return submit(s, job_config(L, beta, J, seed, q, init, sweeps), sweeps, job_id);
}

int sw_server_step(sw_server *s, int64_t n, int64_t *done_ids, int32_t cap, int32_t *ndone) {
    if (!s || !ndone) return fail(SW_EINVAL, "server or ndone is NULL");
    if (n < 0) return fail(SW_EINVAL, "n must be >= 0");
    if (cap < 0 || (cap > 0 && !done_ids)) return fail(SW_EINVAL, "bad done_ids / cap");
    *ndone = 0;
    int rc = srv_device(s);
    if (rc != SW_OK) return rc;
    rc = admit(s);
    if (rc != SW_OK) return rc;
    int64_t left = n;
    while (left > 0 && !s->active.empty()) {
        if (s->dirty) {
            rc = rebuild_active(s);
            if (rc != SW_OK) return rc;
        }
        int64_t k = left;
        for (const Job *j : s->active) k = std::min(k, j->target - j->done);
        for (int64_t i = 0; i < k; ++i)
            for (int g = 0; g < kGroups; ++g) HIP_TRY(swmi::launch_batch_sweep(s->bd[g], s->stream));
        uint64_t sites = 0;
        for (Job *j : s->active) {
            j->done += k;
            sites += (uint64_t)j->cfg.L * (uint64_t)j->cfg.L;
        }
        s->site_updates += sites * (uint64_t)k;
        left -= k;

        // jobs that reached their sweep count: final spins, then leave
        std::vector<Job *> fin, keep;
        for (Job *j : s->active) (j->done == j->target ? fin : keep).push_back(j);
        if (fin.empty()) continue;
        HIP_TRY(hipStreamSynchronize(s->stream));
        swmi::BatchMaps m[kGroups];
        swmi::BatchDev rb[kGroups]{};
        for (Job *j : fin) m[group_of(j->dev)].add((uint32_t)j->slot, j->dev, true);
        set_groups(rb);
        rc = upload_maps(s, m, rb, kGroups);
        if (rc != SW_OK) return rc;
        for (int g = 0; g < kGroups; ++g) HIP_TRY(swmi::launch_batch_resolve(rb[g], s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        for (Job *j : fin) {
            j->state = SW_JOB_DONE;
            s->free_slots.push_back(j->slot);
            j->slot = -1;
            if (*ndone < cap) done_ids[*ndone] = j->id;
            ++*ndone;
        }
        s->active.swap(keep);
        s->dirty = true;
        rc = admit(s);
        if (rc != SW_OK) return rc;
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SW_OK;
}

int sw_server_job_info(sw_server *s, int64_t id, sw_job_info *info) {
    Job *j = nullptr;
    int rc = find_job(s, id, &j);
    if (rc != SW_OK) return rc;
    if (!info) return fail(SW_EINVAL, "info is NULL");
    info->id = j->id;
    info->state = j->state;
    info->L = j->cfg.L;
    info->sweeps_done = j->done;
    info->sweeps_total = j->target;
    info->bytes = j->bytes;
    return SW_OK;
}

int sw_server_job_series(sw_server *s, int64_t id, int64_t first, int64_t count, sw_obs *out) {
    Job *j = nullptr;
    int rc = find_job(s, id, &j);
    if (rc != SW_OK) return rc;
    if (j->state == SW_JOB_QUEUED) return fail(SW_ESTATE, "job has not started");
    if (count < 0 || (count > 0 && !out)) return fail(SW_EINVAL, "bad count or NULL out");
    // The energy and magnetisation of an active job's last record are those
    // of the configuration its last sweep left, measured by the job's next
    // sweep (or by the closing pass when it finishes): until then that
    // record is incomplete and is not handed out.
    const int64_t avail = j->state == SW_JOB_ACTIVE ? j->done - 1 : j->done;
    if (first < 0 || first + count > avail)
        return fail(SW_ERANGE, j->state == SW_JOB_ACTIVE
                                   ? "records requested outside the sweeps run (an active job's last record is "
                                     "complete only after its next sweep)"
                                   : "records requested outside the sweeps run");
    if (count == 0) return SW_OK;
    rc = srv_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(out, j->dev.ring + first, (size_t)count * sizeof(sw_obs), hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_server_job_spins(sw_server *s, int64_t id, int8_t *host, int64_t n) {
    Job *j = nullptr;
    int rc = find_job(s, id, &j);
    if (rc != SW_OK) return rc;
    if (j->state != SW_JOB_DONE) return fail(SW_ESTATE, "spins are available once the job is done");
    if (!host) return fail(SW_EINVAL, "host is NULL");
    if (n != (int64_t)j->cfg.L * j->cfg.L) return fail(SW_ERANGE, "n must equal L*L of the job");
    rc = srv_device(s);
    if (rc != SW_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(host, j->dev.spins[j->done & 1], (size_t)n, hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_server_release(sw_server *s, int64_t id) {
    Job *j = nullptr;
    int rc = find_job(s, id, &j);
    if (rc != SW_OK) return rc;
    if (j->state == SW_JOB_ACTIVE) return fail(SW_ESTATE, "an active job cannot be released");
    if (j->state == SW_JOB_QUEUED) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), j));
    } else {
        rc = srv_device(s);
        if (rc != SW_OK) return rc;
        HIP_TRY(hipStreamSynchronize(s->stream));
        s->pool.release(j->off, j->bytes);
    }
    s->jobs.erase(id);
    delete j;
    return SW_OK;
}

int sw_server_status(sw_server *s, int32_t *queued, int32_t *active, size_t *bytes_used, uint64_t *site_updates) {
    if (!s) return fail(SW_EINVAL, "server is NULL");
    if (queued) *queued = (int32_t)s->queue.size();
    if (active) *active = (int32_t)s->active.size();
    if (bytes_used) *bytes_used = s->pool.used;
    if (site_updates) *site_updates = s->site_updates;
    return SW_OK;
}

void sw_server_destroy(sw_server *s) {
    if (!s) return;
    (void)srv_device(s);
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->jobs) delete kv.second;
    if (s->d_maps) (void)hipFree(s->d_maps);
    if (s->d_devs) (void)hipFree(s->d_devs);
    if (s->own_pool && s->pool_mem) (void)hipFree(s->pool_mem);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
