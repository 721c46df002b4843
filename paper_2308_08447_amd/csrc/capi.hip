// capi.hip -- the extern "C" entry points declared in include/demag.h.
//
// A plan owns, per mesh: the packed FP32 kernel K, the twiddle tables, the two
// spectral workspaces S1 and S2 and (allocated on first use) the RK4 stage
// buffers.  Every entry point validates its arguments on the host before any
// device work is enqueued and reports failures through a status code and a
// thread-local message; nothing throws across the ABI.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <array>
#include <map>
#include <mutex>
#include <vector>

#include "engine.h"

namespace dm {

thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

static bool pow2_or_one(int n) { return n >= 1 && (n & (n - 1)) == 0; }

int make_geometry(int nx, int ny, int nz, Geometry* g) {
    if (nx < 1 || ny < 1 || nz < 1) return fail(DEMAG_EINVAL, "mesh sizes must be >= 1");
    if (!pow2_or_one(nx) || !pow2_or_one(ny) || !pow2_or_one(nz))
        return fail(DEMAG_EUNSUPPORTED, "mesh sizes must be 1 or a power of two");
    if (nx > 2048 || ny > 2048 || nz > 128)
        return fail(DEMAG_EUNSUPPORTED, "mesh too large (nx, ny <= 2048, nz <= 128)");
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->Nx = nx == 1 ? 1 : 2 * nx;
    g->Ny = ny == 1 ? 1 : 2 * ny;
    g->Nz = nz == 1 ? 1 : 2 * nz;
    g->X1 = g->Nx == 1 ? 1 : g->Nx / 2 + 1;
    g->Y1 = g->Ny == 1 ? 1 : g->Ny / 2 + 1;
    g->Z1 = g->Nz == 1 ? 1 : g->Nz / 2 + 1;
    return DEMAG_OK;
}

static int check_mesh(const demag_mesh* m, Geometry* g) {
    if (!m) return fail(DEMAG_EINVAL, "mesh is NULL");
    int rc = make_geometry(m->nx, m->ny, m->nz, g);
    if (rc) return rc;
    const double h[3] = {m->dx, m->dy, m->dz};
    for (double v : h)
        if (!(v > 0.0) || !std::isfinite(v)) return fail(DEMAG_EINVAL, "cell sizes must be finite and > 0");
    return DEMAG_OK;
}

}  // namespace dm

using namespace dm;

struct demag_plan {
    Geometry g;
    double dx, dy, dz;
    uint32_t flags;
    float* K = nullptr;
    float2* tw = nullptr;
    float2* S1 = nullptr;
    float2* S2 = nullptr;   // chunk buffer of xc kx planes; == S1 (xc = X1) when ny == 1
    int xc = 1;             // kx planes S2 holds
    int nch = 1;            // chunks the y/z stages are split into (>= ceil(X1 / xc))
    // RK4 stage buffers (lazily allocated): H, A, B, acc, each 3 N floats
    float* rk = nullptr;
    int device = 0;
    // per-stage event timing (demag_timing_enable)
    int timing_cap = 0;
    std::vector<hipEvent_t> ev[DEMAG_NSTAGES];   // 2 * timing_cap events per stage
    int timing_n[DEMAG_NSTAGES] = {};
    int variant[5] = {1, 1, 1, 1, 1};   // tile-shape variant of each FFT stage
};

struct Tuned {
    std::array<int, 5> variant;
    int nch;
};

// Variants picked by demag_autotune, shared by every plan of the same mesh size in
// this process.
static std::mutex g_tune_mu;
static std::map<std::array<int, 3>, Tuned> g_tuned;

static void free_timing(demag_plan* p) {
    for (int s = 0; s < DEMAG_NSTAGES; ++s) {
        for (hipEvent_t e : p->ev[s]) (void)hipEventDestroy(e);
        p->ev[s].clear();
        p->timing_n[s] = 0;
    }
    p->timing_cap = 0;
}

// Brackets one stage launch with events when timing is enabled.
struct StageTimer {
    demag_plan* p;
    int stage;
    hipStream_t s;
    int slot = -1;
    StageTimer(demag_plan* p_, int stage_, hipStream_t s_) : p(p_), stage(stage_), s(s_) {
        if (p->timing_cap > 0 && p->timing_n[stage] < p->timing_cap) {
            slot = p->timing_n[stage]++;
            (void)hipEventRecord(p->ev[stage][2 * slot], s);
        }
    }
    ~StageTimer() {
        if (slot >= 0) (void)hipEventRecord(p->ev[stage][2 * slot + 1], s);
    }
};

struct atom_plan {
    atom_mesh mesh;
    demag_plan* dp = nullptr;
    float* Mm = nullptr;    // macrocell magnetisation (3 Nm)
    float* Hd0 = nullptr;   // macrocell H_d for S (3 Nm)
    float* Hd1 = nullptr;   // macrocell H_d for S_p (3 Nm)
    float* Sp = nullptr;    // predictor spins (3 N)
    float* f0 = nullptr;    // predictor slope (3 N)
};

// hipMalloc with the HIP error text in the failure message
static int dev_alloc(void** p, size_t bytes, const char* what) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? DEMAG_ENOMEM : DEMAG_EHIP,
                    std::string("hipMalloc(") + what + ", " + std::to_string(bytes) +
                        " B): " + hipGetErrorString(e));
    }
    return DEMAG_OK;
}

static void free_plan(demag_plan* p) {
    if (!p) return;
    free_timing(p);
    (void)hipFree(p->K);
    (void)hipFree(p->tw);
    (void)hipFree(p->S1);
    if (p->S2 != p->S1) (void)hipFree(p->S2);
    (void)hipFree(p->rk);
    delete p;
}

// S2 holds the y/z spectra of a chunk of kx planes.  Its size is capped so a
// chunk's spectra stay resident in the 256 MB Infinity Cache while the chunk's
// y FFT, z convolution and y IFFT run back to back.
static constexpr size_t S2_CHUNK_BYTES = (size_t)128 << 20;

static int s2_planes(const Geometry& g) {
    if (g.ny == 1) return g.X1;
    size_t plane = (size_t)3 * g.nz * g.Ny * sizeof(float2);
    size_t planes = S2_CHUNK_BYTES / plane;
    if (planes < 1) planes = 1;
    return planes >= (size_t)g.X1 ? g.X1 : (int)planes;
}

static size_t plan_bytes(const Geometry& g) {
    size_t b = g.k_elems() * sizeof(float);
    b += (size_t)2 * twiddle_table_length(g) * sizeof(float2);
    b += g.s1_elems() * sizeof(float2);
    if (g.ny > 1) b += (size_t)3 * g.nz * s2_planes(g) * g.Ny * sizeof(float2);
    return b;
}

extern "C" {

const char* demag_last_error(void) { return g_last_error.c_str(); }

size_t demag_plan_bytes(const demag_mesh* mesh, uint32_t flags) {
    Geometry g;
    if (flags != DEMAG_FP32) return 0;
    if (check_mesh(mesh, &g) != DEMAG_OK) return 0;
    return plan_bytes(g);
}

int demag_setup(const demag_mesh* mesh, uint32_t flags, void* stream, demag_plan** out) {
    if (!out) return fail(DEMAG_EINVAL, "out is NULL");
    *out = nullptr;
    Geometry g;
    int rc = check_mesh(mesh, &g);
    if (rc) return rc;
    if (flags != DEMAG_FP32) return fail(DEMAG_EUNSUPPORTED, "unknown flags");
    hipStream_t s = (hipStream_t)stream;
    demag_plan* p = new (std::nothrow) demag_plan();
    if (!p) return fail(DEMAG_ENOMEM, "host allocation failed");
    p->g = g;
    p->dx = mesh->dx;
    p->dy = mesh->dy;
    p->dz = mesh->dz;
    p->flags = flags;
    (void)hipGetDevice(&p->device);
    auto bail = [&](int code) {
        free_plan(p);
        return code;
    };
    if ((rc = dev_alloc((void**)&p->K, g.k_elems() * sizeof(float), "kernel")) ||
        (rc = dev_alloc((void**)&p->S1, g.s1_elems() * sizeof(float2), "S1")))
        return bail(rc);
    p->xc = s2_planes(g);
    p->nch = (g.X1 + p->xc - 1) / p->xc;
    if (g.ny > 1) {
        if ((rc = dev_alloc((void**)&p->S2, (size_t)3 * g.nz * p->xc * g.Ny * sizeof(float2), "S2")))
            return bail(rc);
    } else {
        p->S2 = p->S1;
    }
    int Lmax = twiddle_table_length(g);
    std::vector<float2> tw((size_t)2 * Lmax);
    fill_twiddles(tw.data(), Lmax);
    if ((rc = dev_alloc((void**)&p->tw, tw.size() * sizeof(float2), "twiddles"))) return bail(rc);
    if (hipMemcpyAsync(p->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return bail(fail(DEMAG_EHIP, "twiddle upload failed"));
    rc = compute_kernel(g, mesh->dx, mesh->dy, mesh->dz, p->K, s);
    if (rc) return bail(rc);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find({g.nx, g.ny, g.nz});
        if (it != g_tuned.end()) {
            for (int i = 0; i < 5; ++i) p->variant[i] = it->second.variant[i];
            p->nch = it->second.nch;
        }
    }
    *out = p;
    return DEMAG_OK;
}

int demag_destroy(demag_plan* plan) {
    if (!plan) return fail(DEMAG_EINVAL, "plan is NULL");
    free_plan(plan);
    return DEMAG_OK;
}

}  // extern "C"

static StageArgs stage_args(demag_plan* p, hipStream_t s) {
    StageArgs a{&p->g, p->tw, p->S1, p->S2, p->K, s, {}, p->xc};
    for (int i = 0; i < 5; ++i) a.variant[i] = p->variant[i];
    return a;
}

// x R2C over the whole mesh; then, chunk by chunk of kx planes, y FFT -> z
// convolution -> y IFFT through the chunk buffer; then x C2R.
static int run_field(demag_plan* p, const float* M, float* H, float scale, hipStream_t s) {
    const Geometry& g = p->g;
    StageArgs a = stage_args(p, s);
    int rc;
    {
        StageTimer t(p, DEMAG_STAGE_X_FWD, s);
        if ((rc = launch_x_forward(a, M, scale))) return rc;
    }
    if (g.ny == 1) {
        StageTimer t(p, DEMAG_STAGE_Z_CONV, s);
        if ((rc = launch_z_convolve(a, 0, g.X1))) return rc;
    } else {
        const int per = (g.X1 + p->nch - 1) / p->nch;
        for (int k0 = 0; k0 < g.X1; k0 += per) {
            const int nk = per < g.X1 - k0 ? per : g.X1 - k0;
            {
                StageTimer t(p, DEMAG_STAGE_Y_FWD, s);
                if ((rc = launch_y_forward(a, k0, nk))) return rc;
            }
            {
                StageTimer t(p, DEMAG_STAGE_Z_CONV, s);
                if ((rc = launch_z_convolve(a, k0, nk))) return rc;
            }
            {
                StageTimer t(p, DEMAG_STAGE_Y_INV, s);
                if ((rc = launch_y_inverse(a, k0, nk))) return rc;
            }
        }
    }
    StageTimer t(p, DEMAG_STAGE_X_INV, s);
    return launch_x_inverse(a, H);
}

extern "C" {

int demag_field(demag_plan* plan, const float* M, float* H, void* stream) {
    if (!plan) return fail(DEMAG_EINVAL, "plan is NULL");
    if (!M || !H) return fail(DEMAG_EINVAL, "M and H must be non-NULL device pointers");
    if ((const void*)M == (const void*)H) return fail(DEMAG_EINVAL, "H must not alias M");
    return run_field(plan, M, H, 1.0f, (hipStream_t)stream);
}

int demag_set_variant(demag_plan* plan, int32_t stage, int32_t variant) {
    if (!plan) return fail(DEMAG_EINVAL, "plan is NULL");
    if (stage < 0 || stage > DEMAG_STAGE_X_INV) return fail(DEMAG_EINVAL, "stage must be an FFT stage (0..4)");
    if (variant < 0 || variant >= NVARIANTS) return fail(DEMAG_EINVAL, "variant out of range");
    plan->variant[stage] = variant;
    return DEMAG_OK;
}

int demag_get_variant(demag_plan* plan, int32_t stage, int32_t* variant) {
    if (!plan || !variant) return fail(DEMAG_EINVAL, "NULL argument");
    if (stage < 0 || stage > DEMAG_STAGE_X_INV) return fail(DEMAG_EINVAL, "stage must be an FFT stage (0..4)");
    *variant = plan->variant[stage];
    return DEMAG_OK;
}

int demag_set_chunks(demag_plan* plan, int32_t nchunks) {
    if (!plan) return fail(DEMAG_EINVAL, "plan is NULL");
    const Geometry& g = plan->g;
    const int nmin = (g.X1 + plan->xc - 1) / plan->xc;
    if (nchunks < nmin || nchunks > g.X1)
        return fail(DEMAG_EINVAL, "chunk count out of range [ceil(X1 / planes held), X1]");
    plan->nch = g.ny == 1 ? 1 : nchunks;
    return DEMAG_OK;
}

int demag_get_chunks(demag_plan* plan, int32_t* nchunks) {
    if (!plan || !nchunks) return fail(DEMAG_EINVAL, "NULL argument");
    *nchunks = plan->nch;
    return DEMAG_OK;
}

int demag_autotune(demag_plan* plan, void* stream) {
    if (!plan) return fail(DEMAG_EINVAL, "plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    const Geometry& g = plan->g;
    const size_t n3 = 3 * g.cells();
    float* M = nullptr;
    int rc = dev_alloc((void**)&M, 2 * n3 * sizeof(float), "autotune fields");
    if (rc) return rc;
    float* H = M + n3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(M);
    };
    if (hipMemsetAsync(M, 0, 2 * n3 * sizeof(float), s) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(DEMAG_EHIP, "autotune set-up failed");
    }
    const int saved_cap = plan->timing_cap;
    plan->timing_cap = 0;  // no per-stage events while tuning
    // times `reps` runs of fn on the stream
    auto time_it = [&](auto&& fn, int reps, double* ms_out) -> int {
        int r;
        if ((r = fn())) return r;  // warm-up
        (void)hipEventRecord(e0, s);
        for (int i = 0; i < reps; ++i)
            if ((r = fn())) return r;
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(DEMAG_EHIP, "autotune timing failed");
        *ms_out = ms;
        return DEMAG_OK;
    };
    // 1. tile variants, stage by stage, on the first chunk
    if ((rc = run_field(plan, M, H, 1.0f, s))) { cleanup(); plan->timing_cap = saved_cap; return rc; }
    const int per = (g.X1 + plan->nch - 1) / plan->nch;
    for (int st = 0; st < 5 && !rc; ++st) {
        if ((st == 1 || st == 3) && g.ny == 1) continue;
        double best = 1e30;
        int best_v = plan->variant[st];
        for (int v = 0; v < NVARIANTS && !rc; ++v) {
            plan->variant[st] = v;
            StageArgs a = stage_args(plan, s);
            const int nk = g.ny == 1 ? g.X1 : per;
            auto fn = [&]() -> int {
                switch (st) {
                    case 0: return launch_x_forward(a, M, 1.0f);
                    case 1: return launch_y_forward(a, 0, nk);
                    case 2: return launch_z_convolve(a, 0, nk);
                    case 3: return launch_y_inverse(a, 0, nk);
                    default: return launch_x_inverse(a, H);
                }
            };
            double ms = 0.0;
            rc = time_it(fn, 5, &ms);
            if (!rc && ms < best) {
                best = ms;
                best_v = v;
            }
        }
        plan->variant[st] = best_v;
    }
    // 2. number of chunks, timing the whole evaluation
    if (!rc && g.ny > 1) {
        const int nmin = (g.X1 + plan->xc - 1) / plan->xc;
        double best = 1e30;
        int best_n = plan->nch;
        for (int n = nmin; n <= 8 * nmin && n <= g.X1 && !rc; n *= 2) {
            plan->nch = n;
            double ms = 0.0;
            rc = time_it([&]() { return run_field(plan, M, H, 1.0f, s); }, 3, &ms);
            if (!rc && ms < best) {
                best = ms;
                best_n = n;
            }
        }
        plan->nch = best_n;
    }
    plan->timing_cap = saved_cap;
    cleanup();
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    Tuned t;
    for (int i = 0; i < 5; ++i) t.variant[i] = plan->variant[i];
    t.nch = plan->nch;
    g_tuned[{g.nx, g.ny, g.nz}] = t;
    return DEMAG_OK;
}

int demag_timing_enable(demag_plan* plan, int32_t max_records) {
    if (!plan) return fail(DEMAG_EINVAL, "plan is NULL");
    if (max_records < 0) return fail(DEMAG_EINVAL, "max_records must be >= 0");
    free_timing(plan);
    if (max_records == 0) return DEMAG_OK;
    for (int s = 0; s < DEMAG_NSTAGES; ++s) {
        plan->ev[s].resize((size_t)2 * max_records, nullptr);
        for (auto& e : plan->ev[s]) {
            if (hipEventCreate(&e) != hipSuccess) {
                e = nullptr;
                free_timing(plan);
                return fail(DEMAG_EHIP, "hipEventCreate failed");
            }
        }
    }
    plan->timing_cap = max_records;
    return DEMAG_OK;
}

int demag_timing_read(demag_plan* plan, double* total_ms, int32_t* launches) {
    if (!plan || !total_ms || !launches) return fail(DEMAG_EINVAL, "NULL argument");
    for (int s = 0; s < DEMAG_NSTAGES; ++s) {
        double acc = 0.0;
        for (int i = 0; i < plan->timing_n[s]; ++i) {
            DM_HIP(hipEventSynchronize(plan->ev[s][2 * i + 1]));
            float ms = 0.f;
            DM_HIP(hipEventElapsedTime(&ms, plan->ev[s][2 * i], plan->ev[s][2 * i + 1]));
            acc += ms;
        }
        total_ms[s] = acc;
        launches[s] = plan->timing_n[s];
        plan->timing_n[s] = 0;
    }
    return DEMAG_OK;
}

int demag_get_kernel(demag_plan* plan, float* dst, size_t count, void* stream) {
    if (!plan || !dst) return fail(DEMAG_EINVAL, "plan and dst must be non-NULL");
    size_t n = plan->g.k_elems();
    if (count < n) return fail(DEMAG_EINVAL, "dst too small for the packed kernel");
    DM_HIP(hipMemcpyAsync(dst, plan->K, n * sizeof(float), hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
    return DEMAG_OK;
}

int llg_step(demag_plan* plan, float* m, const llg_params* prm, double dt, int32_t nsteps,
             void* stream) {
    if (!plan || !m || !prm) return fail(DEMAG_EINVAL, "plan, m and params must be non-NULL");
    if (nsteps < 0) return fail(DEMAG_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return fail(DEMAG_EINVAL, "dt must be finite");
    if (!(prm->Ms > 0.0) || !(prm->gamma > 0.0) || !(prm->alpha >= 0.0) || !std::isfinite(prm->A))
        return fail(DEMAG_EINVAL, "invalid LLG parameters (Ms > 0, gamma > 0, alpha >= 0)");
    if (nsteps == 0) return DEMAG_OK;
    hipStream_t s = (hipStream_t)stream;
    const Geometry& g = plan->g;
    const size_t N3 = 3 * g.cells();
    if (!plan->rk) {
        int rc = dev_alloc((void**)&plan->rk, 4 * N3 * sizeof(float), "RK4 buffers");
        if (rc) return rc;
    }
    float* Hd = plan->rk;
    float* bufA = plan->rk + N3;
    float* bufB = plan->rk + 2 * N3;
    float* acc = plan->rk + 3 * N3;
    const double mu0 = 4e-7 * 3.141592653589793238462643383279502884;
    const double cex = 2.0 * prm->A / (mu0 * prm->Ms);
    LLGStageArgs a;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.cx = g.nx > 1 ? (float)(cex / (plan->dx * plan->dx)) : 0.f;
    a.cy = g.ny > 1 ? (float)(cex / (plan->dy * plan->dy)) : 0.f;
    a.cz = g.nz > 1 ? (float)(cex / (plan->dz * plan->dz)) : 0.f;
    for (int d = 0; d < 3; ++d) a.hz[d] = (float)prm->Hzee[d];
    a.gam = (float)(prm->gamma / (1.0 + prm->alpha * prm->alpha));
    a.alpha = (float)prm->alpha;
    a.dt = (float)dt;
    const float Ms = (float)prm->Ms;
    for (int step = 0; step < nsteps; ++step) {
        const float* ms = m;
        float* outs[4] = {bufA, bufB, bufA, m};
        for (int st = 0; st < 4; ++st) {
            int rc = run_field(plan, ms, Hd, Ms, s);
            if (rc) return rc;
            {
                StageTimer t(plan, DEMAG_STAGE_LLG, s);
                rc = launch_llg_stage(a, st, m, ms, Hd, acc, outs[st], s);
            }
            if (rc) return rc;
            ms = outs[st];
        }
    }
    return DEMAG_OK;
}

// ---------------------------------------------------------------- atomistic
static void free_atom(atom_plan* p) {
    if (!p) return;
    if (p->dp) free_plan(p->dp);
    (void)hipFree(p->Mm);
    (void)hipFree(p->Hd0);
    (void)hipFree(p->Hd1);
    (void)hipFree(p->Sp);
    (void)hipFree(p->f0);
    delete p;
}

int atom_setup(const atom_mesh* mesh, uint32_t flags, void* stream, atom_plan** out) {
    if (!out) return fail(DEMAG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mesh) return fail(DEMAG_EINVAL, "mesh is NULL");
    if (mesh->macro < 1) return fail(DEMAG_EINVAL, "macro must be >= 1");
    if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1)
        return fail(DEMAG_EINVAL, "lattice sizes must be >= 1");
    if (mesh->nx % mesh->macro || mesh->ny % mesh->macro || mesh->nz % mesh->macro)
        return fail(DEMAG_EINVAL, "macro must divide every lattice size");
    if (!(mesh->a > 0.0) || !std::isfinite(mesh->a)) return fail(DEMAG_EINVAL, "a must be > 0");
    demag_mesh dm_mesh;
    dm_mesh.nx = mesh->nx / mesh->macro;
    dm_mesh.ny = mesh->ny / mesh->macro;
    dm_mesh.nz = mesh->nz / mesh->macro;
    dm_mesh.dx = dm_mesh.dy = dm_mesh.dz = mesh->a * mesh->macro;
    atom_plan* p = new (std::nothrow) atom_plan();
    if (!p) return fail(DEMAG_ENOMEM, "host allocation failed");
    p->mesh = *mesh;
    int rc = demag_setup(&dm_mesh, flags, stream, &p->dp);
    if (rc) {
        delete p;
        return rc;
    }
    size_t N3 = (size_t)3 * mesh->nx * mesh->ny * mesh->nz;
    size_t M3 = (size_t)3 * dm_mesh.nx * dm_mesh.ny * dm_mesh.nz;
    if ((rc = dev_alloc((void**)&p->Mm, M3 * sizeof(float), "macrocell M")) ||
        (rc = dev_alloc((void**)&p->Hd0, M3 * sizeof(float), "macrocell H_d")) ||
        (rc = dev_alloc((void**)&p->Hd1, M3 * sizeof(float), "macrocell H_d'")) ||
        (rc = dev_alloc((void**)&p->Sp, N3 * sizeof(float), "predictor spins")) ||
        (rc = dev_alloc((void**)&p->f0, N3 * sizeof(float), "predictor slope"))) {
        free_atom(p);
        return rc;
    }
    *out = p;
    return DEMAG_OK;
}

int atom_step(atom_plan* p, float* S, const atom_params* prm, double dt, int32_t nsteps,
              void* stream) {
    if (!p || !S || !prm) return fail(DEMAG_EINVAL, "plan, S and params must be non-NULL");
    if (nsteps < 0) return fail(DEMAG_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return fail(DEMAG_EINVAL, "dt must be finite");
    if (!(prm->mu_s > 0.0) || !(prm->gamma > 0.0) || !(prm->alpha >= 0.0) || !std::isfinite(prm->J))
        return fail(DEMAG_EINVAL, "invalid atomistic parameters (mu_s > 0, gamma > 0, alpha >= 0)");
    hipStream_t s = (hipStream_t)stream;
    const double mu0 = 4e-7 * 3.141592653589793238462643383279502884;
    const double muB = 9.2740100783e-24;
    AtomArgs a;
    a.nx = p->mesh.nx;
    a.ny = p->mesh.ny;
    a.nz = p->mesh.nz;
    a.macro = p->mesh.macro;
    a.cex = (float)(prm->J / (mu0 * muB * prm->mu_s));
    for (int d = 0; d < 3; ++d) a.hz[d] = (float)prm->Hzee[d];
    a.gam = (float)(prm->gamma / (1.0 + prm->alpha * prm->alpha));
    a.alpha = (float)prm->alpha;
    a.dt = (float)dt;
    double ns = (double)p->mesh.macro * p->mesh.macro * p->mesh.macro;
    a.mscale = (float)(prm->mu_s * muB / (p->mesh.a * p->mesh.a * p->mesh.a * ns));
    for (int step = 0; step < nsteps; ++step) {
        int rc;
        if ((rc = launch_macro_average(a, S, p->Mm, s))) return rc;
        if ((rc = run_field(p->dp, p->Mm, p->Hd0, 1.0f, s))) return rc;
        if ((rc = launch_heun_predict(a, S, p->Hd0, p->f0, p->Sp, s))) return rc;
        if ((rc = launch_macro_average(a, p->Sp, p->Mm, s))) return rc;
        if ((rc = run_field(p->dp, p->Mm, p->Hd1, 1.0f, s))) return rc;
        if ((rc = launch_heun_correct(a, S, p->Sp, p->f0, p->Hd1, s))) return rc;
    }
    return DEMAG_OK;
}

int atom_destroy(atom_plan* p) {
    if (!p) return fail(DEMAG_EINVAL, "plan is NULL");
    free_atom(p);
    return DEMAG_OK;
}

}  // extern "C"
