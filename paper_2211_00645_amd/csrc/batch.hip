// batch.hip -- ragged batches of uint16 stacks in one graph launch: either
// one persistent kernel over all jobs (device job table) or one plain paced
// launch per job, whichever the autotuner measures faster on the batch's own
// buffers (on-disk cache of the choice), captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "tune.hpp"
#include "deskew.h"
#include "kernels.hpp"

using namespace dsk;

// One persistent launch: `count` job records from `first` in the table, all
// writing a volume or none (each kind has its own kernel), their tiles
// numbered from 0.
struct SubLaunch {
    int first = 0, count = 0;
    int64_t total = 0;
    int grid = 0;
    bool vol = false;
};

struct dsk_batch {
    int device = 0;
    int n_jobs = 0;
    std::vector<dsk_job> jobs;
    int mode = DSK_BATCH_PERSISTENT;
    std::vector<dsk_tune> job_tunes;     // per-job shapes (DSK_BATCH_PER_JOB_TUNED)
    dsk_tune tune{};
    double best_ms = 0.0;
    SubLaunch subs[2];                   // persistent launches (see encode_table)
    int n_subs = 0;
    JobDev *table_dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

using JobsKernel = void (*)(const JobDev *, int, int64_t);

JobsKernel pick_kernel(const dsk_tune &t, bool vol) {
    return dispatch_tune(t, [vol](auto B, auto P, auto U, auto NT) -> JobsKernel {
        constexpr int b = decltype(B)::value, p = decltype(P)::value, u = decltype(U)::value;
        // launches without a volume only read: no store kind to choose
        if (vol) return k_forward_jobs<b, p, u, decltype(NT)::value, true>;
        return k_forward_jobs<b, p, u, false, false>;
    });
}

int validate_job(const dsk_job &j) {
    if (!j.in || !dims_ok(j.dims) || (!j.vol && !j.psum && !j.pmax)) return DSK_EINVAL;
    if (!j.offsets_dev && !std::isfinite(j.shift_px)) return DSK_EINVAL;
    return check_frame(j.dims, j.origin, j.out_width);
}

// Job table for a launch shape: the jobs that write a volume first, then the
// others, each part numbering its tiles from 0.  Fills one SubLaunch per
// non-empty part (grid still 0) and returns their number, or < 0.
int encode_table(const dsk_job *jobs, int n, const dsk_tune &t, JobDev *out, SubLaunch subs[2]) {
    int ns = 0, k = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const bool vol = pass == 0;
        const int first = k;
        int64_t begin = 0;
        for (int i = 0; i < n; ++i) {
            const dsk_job &j = jobs[i];
            if ((j.vol != nullptr) != vol) continue;
            const bool vec = vec_ok(t, j.dims, j.out_width, j.in, 0, j.vol,
                                    (int64_t)j.dims.rows * j.dims.cols);
            const int64_t tx = tiles_x(j.out_width, t, vec);
            const int64_t eb = edge_blocks(j.dims, j.out_width, t, vec, j.vol != nullptr);
            if (tx > kMaxI32) return -1;
            JobDev r;
            r.in = j.in;
            r.vol = j.vol;
            r.psum = j.psum;
            r.pmax = j.pmax;
            r.offs = j.offsets_dev;
            r.shift = j.shift_px;
            r.origin = (double)j.origin;
            r.W = j.out_width;
            r.tile_begin = begin;
            r.N = j.dims.planes;
            r.R = j.dims.rows;
            r.C = j.dims.cols;
            r.tiles_x = (int32_t)tx;
            r.vec = vec ? 1 : 0;
            r.edge_blocks = (int32_t)eb;
            r.tau256 = 0;
            out[k++] = r;
            begin += tx * j.dims.rows + eb;
            if (begin < 0 || begin > (int64_t(1) << 50)) return -1;
        }
        if (k > first) {
            if (begin <= 0) return -1;
            SubLaunch &sl = subs[ns++];
            sl.first = first;
            sl.count = k - first;
            sl.total = begin;
            sl.grid = 0;
            sl.vol = vol;
        }
    }
    return ns;
}

// Resident workgroups for the persistent grid.
int persistent_grid(const dsk_tune &t, bool vol, int64_t total_tiles) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)pick_kernel(t, vol),
                                                     t.block, 0) != hipSuccess)
        return -1;
    if (per_cu < 1) per_cu = 1;
    if (t.wg_per_cu > 0 && t.wg_per_cu < per_cu) per_cu = t.wg_per_cu;
    int64_t g = (int64_t)cus * per_cu;
    if (g > total_tiles) g = total_tiles;
    if (g < 1) g = 1;
    return (int)g;
}

// Plane pacing of each job: every resident workgroup of the persistent grid
// gets a fair share of the pace, whatever job its current tile belongs to,
// so a tile of job j moves one plane in (job j's plane bytes / its tiles)
// x grid / pace.  Jobs without a volume only read and are not paced.
void set_pacing(JobDev *tab, int n, const dsk_tune &t, int grid) {
    for (int i = 0; i < n; ++i) {
        JobDev &r = tab[i];
        r.tau256 = 0;
        if (!r.vec || !r.vol || t.pace_gbs <= 0) continue;
        const double blocks = (double)r.tiles_x * r.R + r.edge_blocks;
        const double plane_bytes = 2.0 * (double)r.R * r.C + 4.0 * (double)r.R * (double)r.W;
        const double tau = plane_bytes / blocks * (double)grid / ((double)t.pace_gbs * 1e9) *
                           1e8 * 256.0;
        r.tau256 = tau >= 4.0e9 ? 4000000000u : (uint32_t)tau;
    }
}

// Grids and pacing of the table's persistent launches.
int plan_launches(const dsk_tune &t, JobDev *table_host, SubLaunch *subs, int ns) {
    for (int i = 0; i < ns; ++i) {
        SubLaunch &sl = subs[i];
        sl.grid = persistent_grid(t, sl.vol, sl.total);
        if (sl.grid <= 0) return DSK_EHIP;
        set_pacing(table_host + sl.first, sl.count, t, sl.grid);
    }
    return DSK_OK;
}

hipError_t launch_jobs(const JobDev *table, const SubLaunch *subs, int ns, const dsk_tune &t,
                       hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
        const JobDev *tab = table + subs[i].first;
        int n = subs[i].count;
        int64_t total = subs[i].total;
        void *args[] = {(void *)&tab, (void *)&n, (void *)&total};
        e = hipLaunchKernel((const void *)pick_kernel(t, subs[i].vol), dim3(subs[i].grid),
                            dim3(t.block), args, 0, s);
    }
    return e;
}

int log2_bucket(double v) { return v <= 1.0 ? 0 : (int)std::floor(std::log2(v)); }

// Shape class: arch, job count, and log2 buckets of total output voxels
// and mean planes per job.
std::string shape_key(const dsk_job *jobs, int n) {
    double vox = 0.0, planes = 0.0;
    for (int i = 0; i < n; ++i) {
        vox += (double)jobs[i].dims.planes * jobs[i].dims.rows * (double)jobs[i].out_width;
        planes += jobs[i].dims.planes;
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/jobs%d/vox2^%d/planes2^%d", arch_name().c_str(), n,
                  log2_bucket(vox), log2_bucket(planes / n));
    return buf;
}

// Launch shapes the autotuner times.
std::vector<dsk_tune> candidates() {
    std::vector<dsk_tune> c;
    for (int u : {1, 2, 4})
        for (int pace : {0, 5500}) c.push_back(dsk_tune{64, 4, 1, u, 0, pace});
    c.push_back(dsk_tune{256, 8, 1, 2, 0, 0});
    return c;
}

int upload_table(dsk_batch *bt, const dsk_tune &t, hipStream_t s) {
    std::vector<JobDev> host((size_t)bt->n_jobs);
    SubLaunch subs[2];
    const int ns = encode_table(bt->jobs.data(), bt->n_jobs, t, host.data(), subs);
    if (ns <= 0) return DSK_ESHAPE;
    const int st = plan_launches(t, host.data(), subs, ns);
    if (st != DSK_OK) return st;
    hipError_t e = hipMemcpyAsync(bt->table_dev, host.data(), host.size() * sizeof(JobDev),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return DSK_EHIP;
    for (int i = 0; i < ns; ++i) bt->subs[i] = subs[i];
    bt->n_subs = ns;
    return DSK_OK;
}

// Best of `reps` timed launches (ms) of shape t.
int time_shape(dsk_batch *bt, const dsk_tune &t, hipStream_t s, int reps, double *ms) {
    int st = upload_table(bt, t, s);
    if (st != DSK_OK) return st;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return DSK_EHIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return DSK_EHIP;
    }
    double best = 1e300;
    hipError_t e = launch_jobs(bt->table_dev, bt->subs, bt->n_subs, t, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = launch_jobs(bt->table_dev, bt->subs, bt->n_subs, t, s);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float f = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
        if (e == hipSuccess && f < best) best = f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return DSK_EHIP;
    *ms = best;
    return DSK_OK;
}

// Per-job modes: every job as its own plain launch (paced, so each job's
// wavefronts keep to one schedule), in the library default shape or in the
// shape the single-stack tuner picks for the job's frame.
int launch_per_job(const dsk_batch *bt, bool tuned, hipStream_t s) {
    for (size_t i = 0; i < bt->jobs.size(); ++i) {
        const dsk_job &j = bt->jobs[i];
        const dsk_tune &t = tuned ? bt->job_tunes[i] : default_tune(j.vol);
        const int st = launch_forward(j.in, 0, j.dims, j.offsets_dev, j.shift_px, j.origin, j.vol,
                                      j.psum, j.pmax, j.out_width, t, s);
        if (st != DSK_OK) return st;
    }
    return DSK_OK;
}

// The tuner's shape for every job's frame (remembered per frame, so jobs of
// one frame and later batches of it tune once).
int tune_jobs(dsk_batch *bt, hipStream_t s) {
    bt->job_tunes.assign(bt->jobs.size(), kDefaultTune);
    for (size_t i = 0; i < bt->jobs.size(); ++i) {
        const dsk_job &j = bt->jobs[i];
        const int st = dsk_deskew_autotune(j.in, 0, j.dims, j.offsets_dev, j.shift_px, j.origin,
                                           j.vol, j.psum, j.pmax, j.out_width, 3, s,
                                           &bt->job_tunes[i], nullptr);
        if (st != DSK_OK) return st;
    }
    return DSK_OK;
}

int launch_mode(dsk_batch *bt, hipStream_t s) {
    if (bt->mode == DSK_BATCH_PER_JOB) return launch_per_job(bt, false, s);
    if (bt->mode == DSK_BATCH_PER_JOB_TUNED) return launch_per_job(bt, true, s);
    return hip_status(launch_jobs(bt->table_dev, bt->subs, bt->n_subs, bt->tune, s));
}

// Best of `reps` timed runs (ms) of a per-job mode, after one untimed run.
int time_per_job(dsk_batch *bt, bool tuned, hipStream_t s, int reps, double *ms) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return DSK_EHIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return DSK_EHIP;
    }
    double best = 1e300;
    int st = launch_per_job(bt, tuned, s);
    for (int i = 0; i < reps && st == DSK_OK; ++i) {
        if (hipEventRecord(a, s) != hipSuccess) st = DSK_EHIP;
        if (st == DSK_OK) st = launch_per_job(bt, tuned, s);
        if (st == DSK_OK && hipEventRecord(b, s) != hipSuccess) st = DSK_EHIP;
        if (st == DSK_OK && hipEventSynchronize(b) != hipSuccess) st = DSK_EHIP;
        float f = 0.0f;
        if (st == DSK_OK && hipEventElapsedTime(&f, a, b) != hipSuccess) st = DSK_EHIP;
        if (st == DSK_OK && f < best) best = f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != DSK_OK) return st;
    *ms = best;
    return DSK_OK;
}

}  // namespace

extern "C" int dsk_batch_create(const dsk_job *jobs, int n_jobs, const dsk_tune *tune,
                                hipStream_t stream, dsk_batch **out) {
    if (!out || !jobs || n_jobs <= 0) return DSK_EINVAL;
    *out = nullptr;
    if (tune && !tune_ok(*tune)) return DSK_EINVAL;
    for (int i = 0; i < n_jobs; ++i) {
        const int st = validate_job(jobs[i]);
        if (st != DSK_OK) return st;
    }
    dsk_batch *bt = new (std::nothrow) dsk_batch;
    if (!bt) return DSK_ENOMEM;
    bt->n_jobs = n_jobs;
    bt->jobs.assign(jobs, jobs + n_jobs);
    if (hipGetDevice(&bt->device) != hipSuccess) {
        delete bt;
        return DSK_EHIP;
    }
    if (hipMalloc((void **)&bt->table_dev, sizeof(JobDev) * (size_t)n_jobs) != hipSuccess) {
        delete bt;
        return DSK_ENOMEM;
    }
    int st = DSK_OK;
    if (tune) {
        bt->tune = *tune;
        bt->best_ms = 0.0;
    } else {
        const std::string key = shape_key(jobs, n_jobs);
        dsk_tune t{};
        double ms = 0.0;
        int mode = DSK_BATCH_PERSISTENT;
        if (!tune_cache_lookup(key, &t, &ms, &mode)) {
            double best = 1e300;
            for (const dsk_tune &c : candidates()) {
                double m = 0.0;
                st = time_shape(bt, c, stream, 2, &m);
                if (st != DSK_OK) break;
                if (m < best) {
                    best = m;
                    t = c;
                }
            }
            double m = 0.0;
            if (st == DSK_OK) st = time_per_job(bt, false, stream, 2, &m);
            if (st == DSK_OK && m < best) {
                best = m;
                mode = DSK_BATCH_PER_JOB;
            }
            if (st == DSK_OK) st = tune_jobs(bt, stream);
            if (st == DSK_OK) st = time_per_job(bt, true, stream, 2, &m);
            if (st == DSK_OK && m < best) {
                best = m;
                mode = DSK_BATCH_PER_JOB_TUNED;
            }
            ms = best;
            if (st == DSK_OK) tune_cache_store(key, t, ms, mode);
        } else if (mode == DSK_BATCH_PER_JOB_TUNED) {
            st = tune_jobs(bt, stream);
        }
        bt->tune = t;
        bt->best_ms = ms;
        bt->mode = mode;
    }
    if (st == DSK_OK) st = upload_table(bt, bt->tune, stream);
    if (st == DSK_OK) {
        // Capture the persistent launch on a private stream.
        hipStream_t cap = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const int lst = launch_mode(bt, cap);
            e = hipStreamEndCapture(cap, &bt->graph);
            if (lst != DSK_OK) e = hipErrorLaunchFailure;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0);
        if (cap) (void)hipStreamDestroy(cap);
        if (e != hipSuccess) st = DSK_EHIP;
    }
    if (st != DSK_OK) {
        dsk_batch_destroy(bt);
        return st;
    }
    *out = bt;
    return DSK_OK;
}

extern "C" int dsk_batch_launch(dsk_batch *bt, hipStream_t stream) {
    if (!bt || !bt->exec) return DSK_EINVAL;
    return hip_status(hipGraphLaunch(bt->exec, stream));
}

extern "C" int dsk_batch_launch_direct(dsk_batch *bt, hipStream_t stream) {
    if (!bt || !bt->table_dev) return DSK_EINVAL;
    return launch_mode(bt, stream);
}

extern "C" int dsk_batch_get_mode(const dsk_batch *bt, int *mode) {
    if (!bt || !mode) return DSK_EINVAL;
    *mode = bt->mode;
    return DSK_OK;
}

extern "C" int dsk_batch_get_tune(const dsk_batch *bt, dsk_tune *tune, double *ms) {
    if (!bt) return DSK_EINVAL;
    if (tune) *tune = bt->tune;
    if (ms) *ms = bt->best_ms;
    return DSK_OK;
}

extern "C" int dsk_batch_destroy(dsk_batch *bt) {
    if (!bt) return DSK_EINVAL;
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    if (bt->table_dev) (void)hipFree(bt->table_dev);
    delete bt;
    return DSK_OK;
}

extern "C" size_t dsk_jobs_table_bytes(int n_jobs) {
    return n_jobs > 0 ? sizeof(JobDev) * (size_t)n_jobs : 0;
}

extern "C" int dsk_jobs_launch(const dsk_job *jobs, int n_jobs, void *table_host,
                               void *table_dev, size_t table_bytes, const dsk_tune *tune,
                               hipStream_t stream) {
    if (!jobs || n_jobs <= 0 || !table_host || !table_dev) return DSK_EINVAL;
    if (table_bytes < dsk_jobs_table_bytes(n_jobs)) return DSK_ESHAPE;
    bool any_vol = false;
    for (int i = 0; i < n_jobs; ++i) any_vol = any_vol || jobs[i].vol != nullptr;
    dsk_tune t = tune ? *tune : (any_vol ? kDefaultTune : kDefaultProjTune);
    if (!tune_ok(t)) return DSK_EINVAL;
    for (int i = 0; i < n_jobs; ++i) {
        const int st = validate_job(jobs[i]);
        if (st != DSK_OK) return st;
    }
    if (!tune) {
        // wavefronts of different stacks cannot keep one schedule
        for (int i = 1; i < n_jobs; ++i) {
            const dsk_job &a = jobs[0], &b = jobs[i];
            if (a.dims.planes != b.dims.planes || a.dims.rows != b.dims.rows ||
                a.dims.cols != b.dims.cols || a.out_width != b.out_width) {
                t.pace_gbs = 0;
                break;
            }
        }
    }
    JobDev *host = (JobDev *)table_host;
    SubLaunch subs[2];
    const int ns = encode_table(jobs, n_jobs, t, host, subs);
    if (ns <= 0) return DSK_ESHAPE;
    const int st = plan_launches(t, host, subs, ns);
    if (st != DSK_OK) return st;
    hipError_t e = hipMemcpyAsync(table_dev, host, dsk_jobs_table_bytes(n_jobs),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_jobs((const JobDev *)table_dev, subs, ns, t, stream);
    return hip_status(e);
}

#if DSK_CHECK_BOUNDS
int dsk::batch_bounds_violations(unsigned long long *count, bool reset) {
    return read_bounds_violations(count, reset);
}
#endif
