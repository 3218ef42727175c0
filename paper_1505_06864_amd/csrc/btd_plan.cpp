// btd_plan.cpp -- host side of the C ABI (include/btd.h): argument checks,
// partition, workspace layout, and the launch sequence of the decomposition
// method (arXiv:1505.06864, Sec. 2) over the recursion levels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "btd_internal.h"

namespace {

using btd::KArgs;
using btd::Level;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct LevelPlan {
    int N = 0, M = 0, P = 1, nmax = 0;
    std::vector<int> sep;  // P+1 entries: -1, q_0 .. q_{P-2}, N
    size_t off_LU = 0, off_Dw = 0, off_DI = 0, off_W = 0, off_Z = 0, off_Hd = 0, off_Hb = 0, off_Hc = 0;
    size_t off_perm = 0, off_sep = 0;
};

// Equal split: subsystem sizes floor((N-P+1)/P), the first (N-P+1) mod P one row longer.
void equal_split(int N, int P, std::vector<int>& sep) {
    sep.assign(P + 1, 0);
    sep[0] = -1;
    sep[P] = N;
    const int rows = N - (P - 1), base = rows / P, rem = rows % P;
    int pos = 0;
    for (int k = 0; k < P - 1; ++k) {
        pos += base + (k < rem ? 1 : 0);
        sep[k + 1] = pos;
        pos += 1;
    }
}

// Subsystem count of the coupling system (P-1 rows) of a level with P
// subsystems.  k = 0: Eq. SuppMatrM, capped at floor(P/3), at least 2;
// k >= 1: subsystems of about k rows.  1 = Thomas algorithm (fewer than 3
// rows).
int coupling_parts(int P, int M, int R, int k = 0) {
    if (P - 1 < 3) return 1;
    int m;
    if (k <= 0) {
        const double ms = std::sqrt((double)P / 3.0 * (5.0 + 2.0 / (1.0 + (double)R / (double)M)));
        m = (int)std::floor(ms + 0.5);
        if (m > P / 3) m = P / 3;
    } else {
        m = P / (k + 1);   // (Nc + 1) / (k + 1) with Nc = P - 1
    }
    if (m < 2) m = 2;
    return m;
}

// Separator table (-1, separators, N) of the caller's P subsystems: the
// caller's separators or the equal split.
void outer_separators(const btd_desc_t* d, std::vector<int>& sep) {
    if (d->seps && d->P > 1) {
        sep.assign(d->P + 1, 0);
        sep[0] = -1;
        sep[d->P] = d->N;
        for (int k = 0; k < d->P - 1; ++k) sep[k + 1] = d->seps[k];
    } else {
        equal_split(d->N, d->P, sep);
    }
}

bool valid_desc(const btd_desc_t* d) {
    if (!d) return false;
    if (d->N < 1 || d->M < 1 || d->M > BTD_MAX_M || d->P < 1 || d->depth < 0 || d->max_nrhs < 1) return false;
    if (d->coupling_rows < 0 || d->sub_parts < 0) return false;
    if (d->prec != BTD_PREC_F64 && d->prec != BTD_PREC_F32_REFINE) return false;
    if (d->P > 1 && 2 * (int64_t)d->P - 1 > d->N) return false;
    if (d->N > (1 << 24) - 1) return false;
    if (d->seps && d->P > 1) {
        int prev = -1;
        for (int k = 0; k < d->P - 1; ++k) {
            const int q = d->seps[k];
            if (q <= prev + 1 || q < 1 || q > d->N - 2) return false;
            prev = q;
        }
        if (d->N - 1 - prev < 1) return false;
    }
    if (d->sub_parts >= 2) {
        // every subsystem must hold J sub-subsystems: at least 2J - 1 rows
        std::vector<int> sep;
        outer_separators(d, sep);
        for (int k = 0; k < d->P; ++k)
            if (sep[k + 1] - sep[k] - 1 < 2 * d->sub_parts - 1) return false;
        if ((int64_t)d->P * d->sub_parts > (1 << 24)) return false;
    }
    return true;
}

// Level list and factor-workspace layout for a description.
// With sub_parts J >= 2: the separators of the level of P*J subsystems
// (each outer subsystem split equally into J, its J-1 inner separators
// followed by the outer separator), and of the level above it (P
// subsystems of J-1 rows, separated at the outer separators' positions).
void subsystem_levels(const btd_desc_t* d, std::vector<int>& sep0, std::vector<int>& sep1) {
    const int P = d->P, J = d->sub_parts;
    std::vector<int> outer, inner;
    outer_separators(d, outer);
    sep0.assign(1, -1);
    for (int k = 0; k < P; ++k) {
        const int r = outer[k] + 1, nk = outer[k + 1] - outer[k] - 1;
        equal_split(nk, J, inner);
        for (int i = 1; i < J; ++i) sep0.push_back(r + inner[i]);
        sep0.push_back(outer[k + 1]);   // the outer separator (N for the last subsystem)
    }
    sep1.assign(P + 1, 0);
    sep1[0] = -1;
    for (int k = 0; k < P - 1; ++k) sep1[k + 1] = k * J + J - 1;
    sep1[P] = P * J - 1;
}

size_t build_levels(const btd_desc_t* d, std::vector<LevelPlan>& lv) {
    lv.clear();
    size_t off = align_up(sizeof(unsigned long long));  // status word first
    const int J = d->sub_parts >= 2 ? d->sub_parts : 1;
    int N = d->N, P = d->P * J, depth = d->depth;
    const int M = d->M;
    const size_t MM = (size_t)M * M;
    const size_t nblk = (size_t)(M + 31) / 32;
    std::vector<int> sub0, sub1;
    if (J > 1) subsystem_levels(d, sub0, sub1);
    int level = 0;
    while (true) {
        LevelPlan L;
        L.N = N; L.M = M; L.P = P;
        if (J > 1 && level <= 1) {
            L.sep = level == 0 ? sub0 : sub1;
        } else if (level == 0 && d->seps && P > 1) {
            L.sep.assign(P + 1, 0);
            L.sep[0] = -1;
            L.sep[P] = N;
            for (int k = 0; k < P - 1; ++k) L.sep[k + 1] = d->seps[k];
        } else {
            equal_split(N, P, L.sep);
        }
        L.nmax = 0;
        for (int k = 0; k < P; ++k) {
            const int nk = L.sep[k + 1] - L.sep[k] - 1;
            if (nk > L.nmax) L.nmax = nk;
        }
        L.off_LU = off; off = align_up(off + sizeof(double) * N * MM);
        L.off_Dw = off; off = align_up(off + sizeof(double) * P * MM);
        L.off_DI = off; off = align_up(off + sizeof(double) * N * nblk * 2048);
        L.off_W = off; off = align_up(off + sizeof(double) * N * MM * 2);
        if (P > 1) {
            L.off_Z = off; off = align_up(off + sizeof(double) * N * MM * 2);
            L.off_Hd = off; off = align_up(off + sizeof(double) * (P - 1) * MM);
            L.off_Hb = off; off = align_up(off + sizeof(double) * (P - 1) * MM);
            L.off_Hc = off; off = align_up(off + sizeof(double) * (P - 1) * MM);
        }
        L.off_perm = off; off = align_up(off + sizeof(int) * (size_t)N * M);
        L.off_sep = off; off = align_up(off + sizeof(int) * (size_t)(P + 1));
        lv.push_back(L);
        if (P == 1) break;
        const int Nc = P - 1;
        int Pc;
        if (J > 1 && level == 0) {
            Pc = d->P;   // the level above splits at the outer separators
        } else {
            Pc = (depth > 0) ? coupling_parts(P, M, d->max_nrhs, d->coupling_rows) : 1;
            depth = depth > 0 ? depth - 1 : 0;
        }
        N = Nc;
        P = Pc;
        ++level;
    }
    return off;
}

size_t solve_bytes_for(const std::vector<LevelPlan>& lv, int R) {
    size_t off = 0;
    for (const auto& L : lv)
        if (L.P > 1) off = align_up(off + sizeof(double) * (size_t)(L.P - 1) * L.M * R);
    return off > 0 ? off : kAlign;
}

// Side streams (default priority) of each device: the chunks of a level are
// split into groups whose sweeps run on their own streams, forked from and
// joined back to the caller's stream with events, so that one group's LU
// launches overlap the other groups' GEMM and TRSM launches.  The streams
// are created once per device (under a lock) and shared by every host
// thread; the fork and join events belong to the calling thread, so the
// record of one call's fork can never be replaced by another thread's
// record before the side streams have been told to wait on it.
constexpr int kMaxGroups = 4;
constexpr int kMaxDevices = 16;
struct SideStreams {
    std::atomic<bool> ready{false};
    hipStream_t s[kMaxGroups] = {};
};
SideStreams g_side[kMaxDevices];
std::mutex g_side_mu;

struct ThreadEvents {
    bool ready = false;
    hipEvent_t fork = nullptr, join[kMaxGroups] = {}, aux[kMaxGroups + 1] = {};
};
thread_local ThreadEvents t_events[kMaxDevices];

struct StreamPool {
    hipStream_t* s;
    hipEvent_t fork;
    hipEvent_t* join;
    hipEvent_t* aux;   // kMaxGroups + 1 more events of the calling thread
};

// Side streams of the current device and the calling thread's events; false
// when they cannot be created (the caller then runs everything on its own
// stream).
bool stream_pool(StreamPool& out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return false;
    SideStreams& side = g_side[dev];
    if (!side.ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lock(g_side_mu);
        if (!side.ready.load(std::memory_order_relaxed)) {
            for (int g = 0; g < kMaxGroups; ++g)
                if (!side.s[g] && hipStreamCreateWithFlags(&side.s[g], hipStreamNonBlocking) != hipSuccess) return false;
            side.ready.store(true, std::memory_order_release);
        }
    }
    ThreadEvents& ev = t_events[dev];
    if (!ev.ready) {
        if (!ev.fork && hipEventCreateWithFlags(&ev.fork, hipEventDisableTiming) != hipSuccess) return false;
        for (int g = 0; g < kMaxGroups; ++g)
            if (!ev.join[g] && hipEventCreateWithFlags(&ev.join[g], hipEventDisableTiming) != hipSuccess) return false;
        for (int g = 0; g <= kMaxGroups; ++g)
            if (!ev.aux[g] && hipEventCreateWithFlags(&ev.aux[g], hipEventDisableTiming) != hipSuccess) return false;
        ev.ready = true;
    }
    out.s = side.s;
    out.fork = ev.fork;
    out.join = ev.join;
    out.aux = ev.aux;
    return true;
}

// Groups for a level of P chunks: at least 8 chunks per group, at most
// BTD_STREAM_GROUPS (environment, 1..4; default 2: on MI355X two groups
// let one group's LU overlap the other's products and triangular solves,
// more groups starve each other of CUs).
int chunk_groups(int P) {
    static const int cap = [] {
        const char* env = std::getenv("BTD_STREAM_GROUPS");
        const int v = env ? std::atoi(env) : 0;
        return (v >= 1 && v <= kMaxGroups) ? v : 2;
    }();
    int g = P / 8;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

// Event pairs around the launches of one kernel class (measurement only);
// the class is read without the lock on every launch, the event lists are
// guarded.  Pairs released by btd_profile_read go to a free list and are
// recorded again later, so after a first measured pass a launch costs two
// event records and no event creation.
struct Profiler {
    std::atomic<int> cls{-1};
    std::mutex mu;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev, spare;
} g_prof;

bool profile_pair(hipEvent_t& a, hipEvent_t& b) {
    {
        std::lock_guard<std::mutex> lock(g_prof.mu);
        if (!g_prof.spare.empty()) {
            a = g_prof.spare.back().first;
            b = g_prof.spare.back().second;
            g_prof.spare.pop_back();
            return true;
        }
    }
    if (hipEventCreate(&a) != hipSuccess) return false;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return false; }
    return true;
}

hipError_t timed(int cls, hipStream_t s, hipError_t (*fn)(const btd::KArgs&, hipStream_t), const btd::KArgs& ka) {
    if (g_prof.cls.load(std::memory_order_relaxed) != cls) return fn(ka, s);
    hipEvent_t a, b;
    if (!profile_pair(a, b)) return hipErrorUnknown;
    (void)hipEventRecord(a, s);
    hipError_t err = fn(ka, s);
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lock(g_prof.mu);
    g_prof.ev.emplace_back(a, b);
    return err;
}

// Scratch of btd_solve_noalloc: a static device array (one copy per device
// the library runs on, held until the process ends).  In host code its name
// is only a host-side stand-in, so its device address is taken once per
// device with hipGetSymbolAddress (with that device current) and only that
// address is passed to kernels.
static __device__ __align__(256) char scratch[BTD_NOALLOC_SCRATCH_BYTES];
std::atomic<char*> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of the current device's scratch, or nullptr on failure.
char* scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    char* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
        void* addr = nullptr;
        if (hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)) != hipSuccess || !addr) return nullptr;
        p = (char*)addr;
        g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
    return p;
}

// Byte offsets inside the factor workspace: the factor's status word, then
// the status word of the right-hand-side check of the solves.
constexpr size_t kFactorStatus = 0, kSolveStatus = 8;

}  // namespace

struct btd_plan_s {
    btd_desc_t desc;
    std::vector<LevelPlan> levels;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    const double *A = nullptr, *B = nullptr, *C = nullptr;
    unsigned long long* status = nullptr;        // factor status word
    unsigned long long* solve_status = nullptr;  // right-hand-side check of the last solve

    Level level_dev(int l) const {
        const LevelPlan& L = levels[l];
        Level d{};
        if (l == 0) { d.A = A; d.B = B; d.C = C; }
        else {
            const LevelPlan& up = levels[l - 1];
            d.A = (const double*)(ws + up.off_Hd);
            d.B = (const double*)(ws + up.off_Hb);
            d.C = (const double*)(ws + up.off_Hc);
        }
        d.LU = (double*)(ws + L.off_LU);
        d.Dw = (double*)(ws + L.off_Dw);
        d.DI = (double*)(ws + L.off_DI);
        d.W = (double*)(ws + L.off_W);
        d.Z = L.P > 1 ? (double*)(ws + L.off_Z) : nullptr;
        d.Hd = L.P > 1 ? (double*)(ws + L.off_Hd) : nullptr;
        d.Hb = L.P > 1 ? (double*)(ws + L.off_Hb) : nullptr;
        d.Hc = L.P > 1 ? (double*)(ws + L.off_Hc) : nullptr;
        d.perm = (int*)(ws + L.off_perm);
        d.sep = (const int*)(ws + L.off_sep);
        d.N = L.N; d.M = L.M; d.P = L.P; d.level = l;
        return d;
    }
};

namespace {

#define BTD_TRY(x)                                     \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return BTD_ERR_LAUNCH;   \
    } while (0)

// A solve enqueued together with the factor: every level's right-hand-side
// sweep and coupling right-hand side run on their own stream `rs` as soon as
// that level's forward sweep (the LU factors and E) is done, so they overlap
// the level's backward sweep and the factorisation of the deeper levels;
// the recoveries follow on the caller's stream once the whole factor and
// the deepest level's solve are done.
struct FusedSolve {
    int R;
    const double* F;
    double* X;
    char* sws;
    hipStream_t rs;
    hipEvent_t* fw;      // per chunk group: forward sweep done (the calling thread's events)
    hipEvent_t done;     // the right-hand-side stream's last sweep
};

int enqueue_sweep(const btd_plan_s* p, size_t l, int R, const double* F, double* X, hipStream_t s);
int enqueue_couple_rhs(const btd_plan_s* p, size_t l, int R, const double* F, double* X, double* Fc,
                       hipStream_t s, bool recover);
int enqueue_rhs_check(const btd_plan_s* p, int R, const double* F, hipStream_t s);
int enqueue_solve_level(const btd_plan_s* p, size_t l, int R, const double* F, double* X, char* sws,
                        size_t sws_off, hipStream_t s);
int enqueue_factor(btd_plan_s* p, hipStream_t s, FusedSolve* fs = nullptr);

// Offset in the solve workspace of level l's coupling right-hand side (the
// layout enqueue_solve_level walks: one block per level with P > 1).
size_t level_fc_offset(const btd_plan_s* p, size_t l, int R) {
    size_t off = 0;
    for (size_t k = 0; k < l; ++k) {
        const LevelPlan& L = p->levels[k];
        if (L.P > 1) off = align_up(off + sizeof(double) * (size_t)(L.P - 1) * L.M * R);
    }
    return off;
}

// Factor and solve in one launch sequence (FusedSolve); without side streams
// the factor and then the solve on the caller's stream.
int enqueue_factor_solve(btd_plan_s* p, int R, const double* F, double* X, char* sws, hipStream_t s) {
    StreamPool pool{};
    if (!stream_pool(pool)) {
        int rc = enqueue_factor(p, s);
        if (rc != BTD_OK) return rc;
        rc = enqueue_rhs_check(p, R, F, s);
        if (rc != BTD_OK) return rc;
        return enqueue_solve_level(p, 0, R, F, X, sws, 0, s);
    }
    FusedSolve fs{R, F, X, sws, pool.s[kMaxGroups - 1], pool.aux, pool.aux[kMaxGroups]};
    // the right-hand-side stream starts after the caller's earlier work
    BTD_TRY(hipEventRecord(pool.fork, s));
    BTD_TRY(hipStreamWaitEvent(fs.rs, pool.fork, 0));
    int rc = enqueue_rhs_check(p, R, F, fs.rs);
    if (rc != BTD_OK) return rc;
    rc = enqueue_factor(p, s, &fs);
    if (rc != BTD_OK) return rc;
    BTD_TRY(hipEventRecord(fs.done, fs.rs));
    BTD_TRY(hipStreamWaitEvent(s, fs.done, 0));
    // recoveries, deepest level first, on the caller's stream
    for (size_t l = p->levels.size(); l-- > 0;) {
        if (p->levels[l].P == 1) continue;
        const double* Fl = l == 0 ? F : (const double*)(sws + level_fc_offset(p, l - 1, R));
        double* Xl = l == 0 ? X : (double*)(sws + level_fc_offset(p, l - 1, R));
        rc = enqueue_couple_rhs(p, l, R, Fl, Xl, (double*)(sws + level_fc_offset(p, l, R)), s, true);
        if (rc != BTD_OK) return rc;
    }
    return BTD_OK;
}

int enqueue_factor(btd_plan_s* p, hipStream_t s, FusedSolve* fs) {
    BTD_TRY(btd::launch_init_status(p->status, s));
    bool deeper_tables = false;  // separator tables of levels 1.. already enqueued
    for (size_t l = 0; l < p->levels.size(); ++l) {
        const LevelPlan& LP = p->levels[l];
        KArgs ka;
        std::memset(&ka, 0, sizeof(ka));
        ka.L = p->level_dev((int)l);
        ka.status = p->status;
        ka.c0 = 0;
        ka.nc = LP.P;
        ka.lowp = (p->desc.prec == BTD_PREC_F32_REFINE && l == 0) ? 1 : 0;
        if (l == 0 || !deeper_tables)
            BTD_TRY(btd::launch_write_ints((int*)(p->ws + LP.off_sep), LP.sep.data(), LP.P + 1, s));
        // chunk groups, each on its own stream (one group: the caller's stream);
        // with a fused solve the last side stream belongs to the right-hand side
        int G = std::min(chunk_groups(LP.P), fs ? kMaxGroups - 1 : kMaxGroups);
        StreamPool pool{};
        if (G > 1 && !stream_pool(pool)) G = 1;
        hipStream_t gs[kMaxGroups];
        KArgs gk[kMaxGroups];
        for (int g = 0; g < G; ++g) {
            gs[g] = G > 1 ? pool.s[g] : s;
            gk[g] = ka;
            gk[g].c0 = (int)((int64_t)LP.P * g / G);
            gk[g].nc = (int)((int64_t)LP.P * (g + 1) / G) - gk[g].c0;
        }
        if (G > 1) {
            BTD_TRY(hipEventRecord(pool.fork, s));
            for (int g = 0; g < G; ++g) BTD_TRY(hipStreamWaitEvent(gs[g], pool.fork, 0));
            // the caller's stream idles until the groups join: the deeper levels'
            // tables are written there meanwhile instead of ahead of each level
            if (l == 0) {
                for (size_t ll = 1; ll < p->levels.size(); ++ll) {
                    const LevelPlan& LQ = p->levels[ll];
                    BTD_TRY(btd::launch_write_ints((int*)(p->ws + LQ.off_sep), LQ.sep.data(), LQ.P + 1, s));
                }
                deeper_tables = true;
            }
        }
        for (int t = 0; t < LP.nmax; ++t) {
            for (int g = 0; g < G; ++g) {
                gk[g].step = t;
                if (t > 0 || !btd::first_step_reads_inputs(LP.M))
                    BTD_TRY(timed(BTD_KC_FWD_GEMM, gs[g], btd::launch_fwd_gemm, gk[g]));
                BTD_TRY(timed(BTD_KC_GETRF, gs[g], btd::launch_getrf, gk[g]));
                if (!btd::lu_prepares(LP.M)) BTD_TRY(timed(BTD_KC_DIAG_PREP, gs[g], btd::launch_diag_inv, gk[g]));
                BTD_TRY(timed(BTD_KC_GETRS_FACTOR, gs[g], btd::launch_getrs, gk[g]));
            }
        }
        if (fs) {
            // this level's right-hand side needs its forward-sweep factors only
            for (int g = 0; g < G; ++g) {
                BTD_TRY(hipEventRecord(fs->fw[g], gs[g]));
                BTD_TRY(hipStreamWaitEvent(fs->rs, fs->fw[g], 0));
            }
            const double* Fl = l == 0 ? fs->F : (const double*)(fs->sws + level_fc_offset(p, l - 1, fs->R));
            double* Xl = l == 0 ? fs->X : (double*)(fs->sws + level_fc_offset(p, l - 1, fs->R));
            int rc = enqueue_sweep(p, l, fs->R, Fl, Xl, fs->rs);
            if (rc != BTD_OK) return rc;
            if (LP.P > 1) {
                rc = enqueue_couple_rhs(p, l, fs->R, Fl, Xl, (double*)(fs->sws + level_fc_offset(p, l, fs->R)), fs->rs,
                                        false);
                if (rc != BTD_OK) return rc;
            }
        }
        if (LP.P > 1) {
            for (int t = 0; t < LP.nmax; ++t)
                for (int g = 0; g < G; ++g) {
                    gk[g].step = t;
                    // the first backward step only copies the spikes of each chunk's
                    // last row, which the slab solve wrote already (M <= 256)
                    if (t > 0 || !btd::first_step_reads_inputs(LP.M))
                        BTD_TRY(timed(BTD_KC_BWD_GEMM, gs[g], btd::launch_bwd_gemm, gk[g]));
                }
        }
        if (G > 1) {
            for (int g = 0; g < G; ++g) {
                BTD_TRY(hipEventRecord(pool.join[g], gs[g]));
                BTD_TRY(hipStreamWaitEvent(s, pool.join[g], 0));
            }
        }
        if (LP.P > 1) BTD_TRY(timed(BTD_KC_COUPLE, s, btd::launch_couple, ka));
    }
    return BTD_OK;
}

// Right-hand-side sweeps of level l: z on the subsystem rows of X.
int enqueue_sweep(const btd_plan_s* p, size_t l, int R, const double* F, double* X, hipStream_t s) {
    const LevelPlan& LP = p->levels[l];
    KArgs ka;
    std::memset(&ka, 0, sizeof(ka));
    ka.L = p->level_dev((int)l);
    ka.R = R;
    ka.F = F;
    ka.X = X;
    ka.status = p->status;
    ka.c0 = 0;
    ka.nc = LP.P;
    if (btd::rhs_batched(LP.M, R)) {
        for (int t = 0; t < LP.nmax; ++t) {
            ka.step = t;
            BTD_TRY(timed(BTD_KC_RHS_SWEEP, s, btd::launch_rhs_fwd_gemm, ka));
            BTD_TRY(timed(BTD_KC_RHS_SWEEP, s, btd::launch_rhs_getrs, ka));
        }
        for (int t = 0; t + 1 < LP.nmax; ++t) {
            ka.step = t;
            BTD_TRY(timed(BTD_KC_RHS_SWEEP, s, btd::launch_rhs_bwd_gemm, ka));
        }
    } else {
        BTD_TRY(timed(BTD_KC_RHS_SWEEP, s, btd::launch_chunk_solve, ka));
    }
    return BTD_OK;
}

// Coupling right-hand side (Eq. e2311) of level l into Fc, or the recovery
// (Eq. endSolution) of level l from the coupling solution in Fc.
int enqueue_couple_rhs(const btd_plan_s* p, size_t l, int R, const double* F, double* X, double* Fc,
                       hipStream_t s, bool recover) {
    KArgs ka;
    std::memset(&ka, 0, sizeof(ka));
    ka.L = p->level_dev((int)l);
    ka.R = R;
    ka.F = F;
    ka.X = X;
    ka.Fc = Fc;
    ka.status = p->status;
    ka.c0 = 0;
    ka.nc = p->levels[l].P;
    if (recover) BTD_TRY(timed(BTD_KC_RECOVER, s, btd::launch_recover, ka));
    else BTD_TRY(timed(BTD_KC_COUPLE_RHS, s, btd::launch_couple_rhs, ka));
    return BTD_OK;
}

// Solve level l in place on X (which already holds F when l > 0).
int enqueue_solve_level(const btd_plan_s* p, size_t l, int R, const double* F, double* X, char* sws,
                        size_t sws_off, hipStream_t s) {
    const LevelPlan& LP = p->levels[l];
    int rc = enqueue_sweep(p, l, R, F, X, s);
    if (rc != BTD_OK) return rc;
    if (LP.P > 1) {
        double* Fc = (double*)(sws + sws_off);
        const size_t next = align_up(sws_off + sizeof(double) * (size_t)(LP.P - 1) * LP.M * R);
        rc = enqueue_couple_rhs(p, l, R, F, X, Fc, s, false);
        if (rc != BTD_OK) return rc;
        rc = enqueue_solve_level(p, l + 1, R, Fc, Fc, sws, next, s);
        if (rc != BTD_OK) return rc;
        rc = enqueue_couple_rhs(p, l, R, F, X, Fc, s, true);
        if (rc != BTD_OK) return rc;
    }
    return BTD_OK;
}

// The check of the right-hand side every solve starts with (non-finite
// entries of F, reported by btd_get_solve_info).
int enqueue_rhs_check(const btd_plan_s* p, int R, const double* F, hipStream_t s) {
    BTD_TRY(btd::launch_init_status(p->solve_status, s));
    BTD_TRY(btd::launch_check_finite(F, p->desc.N, p->desc.M, R, p->solve_status, s));
    return BTD_OK;
}

// A status word (level, row, col, code) read back from the device.
int read_status(const btd_plan_s* p, const unsigned long long* word, int32_t* status, int32_t* block_row,
                int32_t* col) {
    unsigned long long key = ~0ULL;
    if (hipMemcpy(&key, word, sizeof(key), hipMemcpyDeviceToHost) != hipSuccess) return BTD_ERR_LAUNCH;
    int st = BTD_OK, row = -1, c = -1;
    if (key != ~0ULL) {
        const int level = (int)(key >> 56);
        row = (int)((key >> 32) & 0xffffff);
        c = (int)((key >> 8) & 0xffffff);
        st = (int)(key & 0xff);
        // map a coupling-system row back to the separator row of the level above
        for (int l = level; l > 0; --l) row = p->levels[l - 1].sep[row + 1];
    }
    if (status) *status = st;
    if (block_row) *block_row = row;
    if (col) *col = c;
    return BTD_OK;
}

int ensure_configured() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] { err = btd::configure_kernels(); });
    return err == hipSuccess ? BTD_OK : BTD_ERR_LAUNCH;
}

}  // namespace

#ifdef BTD_PHASE_TIMING
namespace btd {
hipError_t read_phase_times(unsigned long long* out);
}
#endif

extern "C" {

int btd_workspace_bytes(const btd_desc_t* desc, size_t* factor_ws, size_t* solve_ws) {
    if (!valid_desc(desc)) return -1;
    std::vector<LevelPlan> lv;
    const size_t f = build_levels(desc, lv);
    if (factor_ws) *factor_ws = f;
    if (solve_ws) *solve_ws = solve_bytes_for(lv, desc->max_nrhs);
    return BTD_OK;
}

}  // extern "C"

namespace {

// Checks btd_factor's arguments and builds the host plan (nothing enqueued).
int new_plan(const btd_desc_t* desc, const double* A, const double* B, const double* C, void* factor_ws,
             size_t factor_bytes, btd_plan_t* out, btd_plan_s** plan) {
    if (!valid_desc(desc)) return -1;
    if (!A) return -2;
    if (!B) return -3;
    if (!C) return -4;
    if (!out) return -8;
    *out = nullptr;
    std::vector<LevelPlan> lv;
    const size_t need = build_levels(desc, lv);
    if (!factor_ws || ((uintptr_t)factor_ws % kAlign) != 0) return -5;
    if (factor_bytes < need) return -6;
    int rc = ensure_configured();
    if (rc != BTD_OK) return rc;
    btd_plan_s* p = new (std::nothrow) btd_plan_s;
    if (!p) return BTD_ERR_LAUNCH;
    p->desc = *desc;
    p->desc.seps = nullptr;
    p->levels = std::move(lv);
    p->ws = (char*)factor_ws;
    p->ws_bytes = factor_bytes;
    p->A = A; p->B = B; p->C = C;
    p->status = (unsigned long long*)((char*)factor_ws + kFactorStatus);
    p->solve_status = (unsigned long long*)((char*)factor_ws + kSolveStatus);
    *plan = p;
    return BTD_OK;
}

}  // namespace

extern "C" {

int btd_factor(const btd_desc_t* desc, const double* A, const double* B, const double* C, void* factor_ws,
               size_t factor_bytes, void* stream, btd_plan_t* out) {
    btd_plan_s* p = nullptr;
    int rc = new_plan(desc, A, B, C, factor_ws, factor_bytes, out, &p);
    if (rc != BTD_OK) return rc;
    rc = enqueue_factor(p, (hipStream_t)stream);
    if (rc != BTD_OK) { delete p; return rc; }
    *out = p;
    return BTD_OK;
}

int btd_factor_solve(const btd_desc_t* desc, const double* A, const double* B, const double* C, void* factor_ws,
                     size_t factor_bytes, int32_t nrhs, const double* F, double* X, void* solve_ws,
                     size_t solve_bytes, void* stream, btd_plan_t* out) {
    if (desc && valid_desc(desc) && (nrhs < 1 || nrhs > desc->max_nrhs)) return -7;
    if (!F) return -9;
    if (!X) return -10;
    btd_plan_s* p = nullptr;
    int rc = new_plan(desc, A, B, C, factor_ws, factor_bytes, out, &p);
    if (rc != BTD_OK) return rc;
    if (!solve_ws || ((uintptr_t)solve_ws % kAlign) != 0) { delete p; return -11; }
    if (solve_bytes < solve_bytes_for(p->levels, nrhs)) { delete p; return -12; }
    rc = enqueue_factor_solve(p, nrhs, F, X, (char*)solve_ws, (hipStream_t)stream);
    if (rc != BTD_OK) { delete p; return rc; }
    *out = p;
    return BTD_OK;
}

int btd_solve(btd_plan_t plan, int32_t nrhs, const double* F, double* X, void* solve_ws, size_t solve_bytes,
              void* stream) {
    if (!plan) return -1;
    if (nrhs < 1 || nrhs > plan->desc.max_nrhs) return -2;
    if (!F) return -3;
    if (!X) return -4;
    const size_t need = solve_bytes_for(plan->levels, nrhs);
    if (!solve_ws || ((uintptr_t)solve_ws % kAlign) != 0) return -5;
    if (solve_bytes < need) return -6;
    int rc = ensure_configured();
    if (rc != BTD_OK) return rc;
    rc = enqueue_rhs_check(plan, nrhs, F, (hipStream_t)stream);
    if (rc != BTD_OK) return rc;
    return enqueue_solve_level(plan, 0, nrhs, F, X, (char*)solve_ws, 0, (hipStream_t)stream);
}

// Workspace of btd_solve_refine: the solve workspace, the residual vector
// [N][M][R], the residual kernels' partial sums and the R column norms.
struct RefineLayout {
    size_t solve, rvec, part, norms, total;
};
RefineLayout refine_layout(const btd_plan_s* p, int R) {
    RefineLayout L{};
    const int N = p->desc.N, M = p->desc.M;
    L.solve = 0;
    L.rvec = align_up(solve_bytes_for(p->levels, R));
    L.part = L.rvec + align_up(sizeof(double) * (size_t)N * M * R);
    L.norms = L.part + align_up(btd_residual_work_bytes(N, M, R));
    L.total = L.norms + align_up(sizeof(double) * (size_t)R);
    return L;
}

size_t btd_refine_work_bytes(btd_plan_t plan, int32_t nrhs) {
    if (!plan || nrhs < 1 || nrhs > plan->desc.max_nrhs) return 0;
    return refine_layout(plan, nrhs).total;
}

int btd_solve_refine(btd_plan_t plan, int32_t nrhs, const double* F, double* X, void* work, size_t work_bytes,
                     double tol, int32_t max_iter, int32_t* iters, double* resid, void* stream) {
    if (!plan) return -1;
    if (nrhs < 1 || nrhs > plan->desc.max_nrhs) return -2;
    if (!F) return -3;
    if (!X || X == F) return -4;
    if (!work || ((uintptr_t)work % kAlign) != 0) return -5;
    const RefineLayout lay = refine_layout(plan, nrhs);
    if (work_bytes < lay.total) return -6;
    if (!(tol > 0.0) || max_iter < 0) return -7;
    int rc = ensure_configured();
    if (rc != BTD_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)work;
    double* rv = (double*)(w + lay.rvec);
    double* part = (double*)(w + lay.part);
    double* norms = (double*)(w + lay.norms);
    const int N = plan->desc.N, M = plan->desc.M, R = nrhs;
    const size_t n = (size_t)N * M * R;
    rc = enqueue_rhs_check(plan, R, F, s);
    if (rc != BTD_OK) return rc;
    rc = enqueue_solve_level(plan, 0, R, F, X, w + lay.solve, 0, s);
    if (rc != BTD_OK) return rc;
    std::vector<double> h(R);
    int it = 0;
    double worst = 0.0;
    while (true) {
        hipEvent_t ea = nullptr, eb = nullptr;
        if (g_prof.cls.load(std::memory_order_relaxed) == BTD_KC_RESIDUAL) {
            if (!profile_pair(ea, eb)) return BTD_ERR_LAUNCH;
            (void)hipEventRecord(ea, s);
        }
        BTD_TRY(btd::launch_residual(N, M, R, plan->A, plan->B, plan->C, X, F, norms, part, s, rv));
        if (ea) {
            (void)hipEventRecord(eb, s);
            std::lock_guard<std::mutex> lock(g_prof.mu);
            g_prof.ev.emplace_back(ea, eb);
        }
        BTD_TRY(hipMemcpyAsync(h.data(), norms, sizeof(double) * R, hipMemcpyDeviceToHost, s));
        BTD_TRY(hipStreamSynchronize(s));
        worst = 0.0;
        for (int c = 0; c < R; ++c) worst = std::isnan(h[c]) || h[c] > worst ? h[c] : worst;
        if (worst <= tol || it >= max_iter || std::isnan(worst)) break;
        // correction: D = A^{-1} r (in place on the residual vector), X += D
        rc = enqueue_solve_level(plan, 0, R, rv, rv, w + lay.solve, 0, s);
        if (rc != BTD_OK) return rc;
        BTD_TRY(btd::launch_add(X, rv, n, s));
        ++it;
    }
    if (iters) *iters = it;
    if (resid) *resid = worst;
    return worst <= tol ? BTD_OK : BTD_ERR_NOT_CONVERGED;
}

int btd_solve_noalloc(btd_plan_t plan, int32_t nrhs, const double* F, double* X, void* stream) {
    if (!plan) return -1;
    if (nrhs < 1 || nrhs > plan->desc.max_nrhs) return -2;
    if (!F) return -3;
    if (!X) return -4;
    if (solve_bytes_for(plan->levels, nrhs) > BTD_NOALLOC_SCRATCH_BYTES) return BTD_ERR_SCRATCH;
    int rc = ensure_configured();
    if (rc != BTD_OK) return rc;
    char* ws = scratch_ptr();
    if (!ws) return BTD_ERR_LAUNCH;
    hipStream_t s = (hipStream_t)stream;
    rc = enqueue_rhs_check(plan, nrhs, F, s);
    if (rc != BTD_OK) return rc;
    return enqueue_solve_level(plan, 0, nrhs, F, X, ws, 0, s);
}

int btd_solve_local(btd_plan_t plan, int32_t nrhs, const double* F, double* X, double* Fhat, void* stream) {
    if (!plan) return -1;
    if (nrhs < 1 || nrhs > plan->desc.max_nrhs) return -2;
    if (!F) return -3;
    if (!X) return -4;
    if (plan->levels[0].P > 1 && !Fhat) return -5;
    int rc = ensure_configured();
    if (rc != BTD_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = enqueue_rhs_check(plan, nrhs, F, s);
    if (rc != BTD_OK) return rc;
    rc = enqueue_sweep(plan, 0, nrhs, F, X, s);
    if (rc != BTD_OK || plan->levels[0].P == 1) return rc;
    return enqueue_couple_rhs(plan, 0, nrhs, F, X, Fhat, s, false);
}

int btd_solve_finish(btd_plan_t plan, int32_t nrhs, const double* H, double* X, void* stream) {
    if (!plan) return -1;
    if (nrhs < 1 || nrhs > plan->desc.max_nrhs) return -2;
    if (plan->levels[0].P > 1 && !H) return -3;
    if (!X) return -4;
    if (plan->levels[0].P == 1) return BTD_OK;
    int rc = ensure_configured();
    if (rc != BTD_OK) return rc;
    return enqueue_couple_rhs(plan, 0, nrhs, nullptr, X, const_cast<double*>(H), (hipStream_t)stream, true);
}

int btd_get_solve_info(btd_plan_t plan, int32_t* status, int32_t* block_row, int32_t* col) {
    if (!plan) return -1;
    return read_status(plan, plan->solve_status, status, block_row, col);
}

int btd_plan_level_arrays(btd_plan_t plan, int32_t level, btd_level_arrays_t* out) {
    if (!plan || !out || level < 0 || level >= (int)plan->levels.size()) return -1;
    const Level d = plan->level_dev(level);
    out->N = d.N;
    out->M = d.M;
    out->P = d.P;
    out->A = d.A;
    out->B = d.B;
    out->C = d.C;
    out->W = d.W;
    out->Z = d.Z;
    out->Hd = d.Hd;
    out->Hb = d.Hb;
    out->Hc = d.Hc;
    out->sep = d.sep;
    return BTD_OK;
}

int btd_solve_batch(int32_t count, const btd_plan_t* plans, const int32_t* nrhs, const double* const* F,
                    double* const* X, void* solve_ws, size_t solve_bytes, void* stream) {
    if (count < 0 || (count > 0 && (!plans || !nrhs || !F || !X))) return -1;
    for (int s = 0; s < count; ++s) {
        if (!plans[s] || nrhs[s] < 1 || nrhs[s] > plans[s]->desc.max_nrhs || !F[s] || !X[s]) return -(1000 + s);
    }
    if (count > 0) {
        size_t need = 0;
        for (int s = 0; s < count; ++s) {
            const size_t b = solve_bytes_for(plans[s]->levels, nrhs[s]);
            if (b > need) need = b;
        }
        if (!solve_ws || ((uintptr_t)solve_ws % kAlign) != 0 || solve_bytes < need) return -6;
    }
    if (count == 0) return BTD_OK;
    int rc0 = ensure_configured();
    if (rc0 != BTD_OK) return rc0;
    hipStream_t s0 = (hipStream_t)stream;
    for (int s = 0; s < count; ++s) {
        int rc = enqueue_rhs_check(plans[s], nrhs[s], F[s], s0);
        if (rc != BTD_OK) return rc;
    }
    // with room for k solves in solve_ws, up to k of them run side by side on
    // the library's side streams, each in its own slice of the workspace
    size_t need = 0;
    for (int s = 0; s < count; ++s) need = std::max(need, solve_bytes_for(plans[s]->levels, nrhs[s]));
    const size_t slice = align_up(need);
    int lanes = (int)std::min<size_t>({solve_bytes / slice, (size_t)kMaxGroups, (size_t)count});
    StreamPool pool{};
    if (lanes > 1 && !stream_pool(pool)) lanes = 1;
    if (lanes == 1) {
        for (int s = 0; s < count; ++s) {
            int rc = enqueue_solve_level(plans[s], 0, nrhs[s], F[s], X[s], (char*)solve_ws, 0, s0);
            if (rc != BTD_OK) return rc;
        }
        return BTD_OK;
    }
    BTD_TRY(hipEventRecord(pool.fork, s0));
    for (int g = 0; g < lanes; ++g) BTD_TRY(hipStreamWaitEvent(pool.s[g], pool.fork, 0));
    for (int s = 0; s < count; ++s) {
        const int g = s % lanes;
        int rc = enqueue_solve_level(plans[s], 0, nrhs[s], F[s], X[s], (char*)solve_ws + (size_t)g * slice, 0,
                                     pool.s[g]);
        if (rc != BTD_OK) return rc;
    }
    for (int g = 0; g < lanes; ++g) {
        BTD_TRY(hipEventRecord(pool.join[g], pool.s[g]));
        BTD_TRY(hipStreamWaitEvent(s0, pool.join[g], 0));
    }
    return BTD_OK;
}

size_t btd_residual_work_bytes(int32_t N, int32_t M, int32_t R) {
    if (N < 1 || M < 1 || R < 1) return 0;
    return sizeof(double) * 2 * btd::residual_parts(N, M, R) * R;
}

int btd_residual(int32_t N, int32_t M, int32_t R, const double* A, const double* B, const double* C,
                 const double* X, const double* F, double* out, void* work, void* stream) {
    if (N < 1 || M < 1 || R < 1 || N > 65535 * 1024) return -1;
    if (!A) return -4;
    if (!B) return -5;
    if (!C) return -6;
    if (!X) return -7;
    if (!F) return -8;
    if (!out) return -9;
    if (!work) return -10;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    if (g_prof.cls.load(std::memory_order_relaxed) == BTD_KC_RESIDUAL) {
        if (!profile_pair(a, b)) return BTD_ERR_LAUNCH;
        (void)hipEventRecord(a, s);
    }
    BTD_TRY(btd::launch_residual(N, M, R, A, B, C, X, F, out, (double*)work, s));
    if (a) {
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lock(g_prof.mu);
        g_prof.ev.emplace_back(a, b);
    }
    return BTD_OK;
}

int btd_get_info(btd_plan_t plan, int32_t* status, int32_t* block_row, int32_t* col) {
    if (!plan) return -1;
    return read_status(plan, plan->status, status, block_row, col);
}

int btd_plan_separators(btd_plan_t plan, int32_t* seps_out) {
    if (!plan || !seps_out) return -1;
    const LevelPlan& L = plan->levels[0];
    const int J = plan->desc.sub_parts >= 2 ? plan->desc.sub_parts : 1;
    for (int k = 0; k < plan->desc.P - 1; ++k) seps_out[k] = L.sep[(k + 1) * J];
    return BTD_OK;
}

int btd_plan_level_parts(btd_plan_t plan, int32_t level) {
    if (!plan || level < 0 || level >= (int)plan->levels.size()) return -1;
    return plan->levels[level].P;
}

int btd_default_separators(int32_t N, int32_t P, int32_t* seps_out) {
    if (N < 1 || P < 1 || (P > 1 && 2 * (int64_t)P - 1 > N) || (P > 1 && !seps_out)) return -1;
    std::vector<int> sep;
    equal_split(N, P, sep);
    for (int k = 0; k < P - 1; ++k) seps_out[k] = sep[k + 1];
    return BTD_OK;
}

int btd_balanced_separators(int32_t N, int32_t P, double alpha, double beta, int32_t* seps_out) {
    if (N < 1 || P < 1 || (P > 1 && 2 * (int64_t)P - 1 > N) || (P > 1 && !seps_out)) return -1;
    if (!(alpha >= 1.0 && alpha <= 64.0) || !(beta >= 1.0 && beta <= 64.0)) return -1;
    if (P == 1) return BTD_OK;
    // subsystem rows T = N - (P-1); the middle size x = T / (P - 2 + alpha + beta),
    // the first alpha x and the last beta x (rounded), every subsystem >= 1 row
    const int T = N - (P - 1);
    const double x = T / (P - 2 + alpha + beta);
    std::vector<int> n(P, 0);
    int first = std::max(1, (int)std::lround(alpha * x)), last = std::max(1, (int)std::lround(beta * x));
    if (P == 2) {
        first = std::min(first, T - 1);
        last = T - first;
    } else {
        while (T - first - last < P - 2) {   // room for one row per middle subsystem
            if (first >= last) --first;
            else --last;
        }
        const int rest = T - first - last, q = rest / (P - 2), r = rest % (P - 2);
        for (int k = 1; k < P - 1; ++k) n[k] = q + (k - 1 < r ? 1 : 0);
    }
    n[0] = first;
    n[P - 1] = last;
    int pos = 0;
    for (int k = 0; k < P - 1; ++k) {
        pos += n[k];
        seps_out[k] = pos;
        pos += 1;
    }
    return BTD_OK;
}

int btd_default_coupling_parts(int32_t P, int32_t M, int32_t R) {
    if (P < 1 || M < 1 || R < 1) return -1;
    return coupling_parts(P, M, R);
}

int btd_coupling_parts(int32_t P, int32_t M, int32_t R, int32_t coupling_rows) {
    if (P < 1 || M < 1 || R < 1 || coupling_rows < 0) return -1;
    return coupling_parts(P, M, R, coupling_rows);
}

int btd_profile_enable(int32_t kernel_class) {
    if (kernel_class < -1 || kernel_class >= BTD_KC_COUNT) return -1;
    g_prof.cls.store(kernel_class);
    return BTD_OK;
}

int btd_profile_read(double* total_ms, int64_t* launches) {
    double tot = 0.0;
    int64_t n = 0;
    int rc = BTD_OK;
    std::lock_guard<std::mutex> lock(g_prof.mu);
    for (auto& pr : g_prof.ev) {
        float ms = 0.0f;
        if (hipEventSynchronize(pr.second) != hipSuccess || hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
            rc = BTD_ERR_LAUNCH;
        tot += ms;
        ++n;
        g_prof.spare.push_back(pr);
    }
    g_prof.ev.clear();
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    return rc;
}

#ifdef BTD_PHASE_TIMING
int btd_debug_phase_times(unsigned long long* out) { return btd::read_phase_times(out) == hipSuccess ? 0 : 3; }
#endif

void btd_plan_destroy(btd_plan_t plan) { delete plan; }

const char* btd_status_string(int code) {
    switch (code) {
        case BTD_OK: return "ok";
        case BTD_ERR_SINGULAR: return "exactly zero pivot in the LU of a diagonal block";
        case BTD_ERR_NONFINITE: return "non-finite pivot in the LU of a diagonal block";
        case BTD_ERR_LAUNCH: return "HIP launch or copy failed";
        case BTD_ERR_SCRATCH: return "solve needs more scratch than the static buffer of btd_solve_noalloc";
        case BTD_ERR_NOT_CONVERGED: return "iterative refinement did not reach the tolerance";
        default: return code < 0 ? "invalid argument" : "unknown status";
    }
}

}  // extern "C"
