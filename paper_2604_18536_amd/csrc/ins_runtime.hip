// Runtime behind the C ABI of include/ins.h: context, FFT plans, workspace,
// the forward and reverse RK4 schedules, error state and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ins.h"
#include "ins_internal.hpp"

using ins::cd;

namespace {

thread_local std::string g_last_error;

struct InsError {
    ins_status st;
    std::string msg;
};

[[noreturn]] void raise(ins_status st, const std::string& msg) { throw InsError{st, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) raise(INS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int kMaxLen = 4096;
constexpr int kBlockHost = 256; // must match kBlock
constexpr size_t kMaxLds = 98304;  // LDS budget of one FFT workgroup
constexpr size_t kCuLds = 163840;  // LDS of one gfx950 compute unit

bool factor(int n, std::vector<int>& rad) {
    rad.clear();
    int m = n, e2 = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++e2;
    }
    while (e2 >= 3) {
        rad.push_back(8);
        e2 -= 3;
    }
    if (e2 == 2) rad.push_back(4);
    if (e2 == 1) rad.push_back(2);
    for (int q : {7, 5, 3}) {
        while (m % q == 0) {
            rad.push_back(q);
            m /= q;
        }
    }
    if (m != 1) return false;
    std::sort(rad.begin(), rad.end(), std::greater<int>());
    return static_cast<int>(rad.size()) <= ins::kMaxStages;
}

// Twiddles exp(-2 pi i q k / (p R)), k < p, 1 <= q < R, for every stage
// (the x passes read these), then the roots W_n^j = exp(-2 pi i j / n), j < n
// (every stage twiddle is the root j = q k n / (p R); the strided passes read
// these). Angles are reduced exactly in integers and evaluated in long double.
void build_twiddles(int n, const std::vector<int>& rad, std::vector<cd>& tw, ins::FftPlan& pl) {
    const long double two_pi = 6.283185307179586476925286766559005768L;
    pl.n = n;
    pl.nst = static_cast<int>(rad.size());
    int p = 1;
    for (int s = 0; s < pl.nst; ++s) {
        const int R = rad[s];
        pl.rad[s] = R;
        pl.tw_off[s] = static_cast<int>(tw.size());
        const long long pr = static_cast<long long>(p) * R;
        for (int k = 0; k < p; ++k) {
            for (int q = 1; q < R; ++q) {
                const long long m = (static_cast<long long>(q) * k) % pr;
                const long double ang = -two_pi * static_cast<long double>(m) / static_cast<long double>(pr);
                tw.push_back(cd{static_cast<double>(cosl(ang)), static_cast<double>(sinl(ang))});
            }
        }
        p *= R;
    }
    pl.rt_off = static_cast<int>(tw.size());
    for (int j = 0; j < n; ++j) {
        const long double ang = -two_pi * static_cast<long double>(j) / static_cast<long double>(n);
        tw.push_back(cd{static_cast<double>(cosl(ang)), static_cast<double>(sinl(ang))});
    }
}

// LDS of one FFT workgroup: nl lines of stride nl + pad, plus `extra` bytes
// (the roots and eigenvalues a pass keeps next to them).
size_t fft_lds(const ins::FftPlan& pl, int nl, int pad, size_t extra) {
    return static_cast<size_t>(nl + pad) * pl.n * sizeof(cd) + extra;
}

// Largest power-of-two line batch (<= maxl) whose every stage fits the
// per-thread register budget vm with nth threads and whose LDS fits the budget.
int lines_for(const ins::FftPlan& pl, int maxl, int vm, int pad, int nth, size_t extra) {
    for (int nl = maxl; nl >= 1; nl >>= 1) {
        if (fft_lds(pl, nl, pad, extra) > kMaxLds) continue;
        bool ok = true;
        for (int s = 0; s < pl.nst; ++s) {
            const int R = pl.rad[s];
            const int bmax = vm / R > 0 ? vm / R : 1;
            const long long nb = static_cast<long long>(nl) * (pl.n / R);
            if (nb > static_cast<long long>(bmax) * nth) ok = false;
        }
        if (ok) {
            int l = 0;
            while ((1 << l) < nl) ++l;
            return l;
        }
    }
    return -1;
}

// Pick the workgroup shape: 8 complex values per thread and 256 threads keep
// occupancy high and are preferred; when that gives batches of fewer than
// `want` lines, a wider workgroup with 8 values per thread (`wide` threads),
// then (the x passes, `wide10`) 10 values per thread with that many threads,
// and only then 16 values per thread with 256 threads. The x passes of n_x =
// 840 (8 rows of 420, radices 7, 5, 4, 3) take 10 values x 512 threads: 128
// registers, 4 waves per SIMD instead of the 2 that 16 values x 256 threads
// (211 registers) left (840^3: x forward 4.96 -> 4.34 ms, x inverse 3.08 ->
// 2.48 ms; the strided passes gained nothing from that shape, their z solve
// lost 8%). The LDS stride is
// padded when that does not narrow the batch and, with `occ`, does not cost a
// workgroup per CU either (the strided passes). `extra`: LDS bytes the pass
// keeps beside the lines. Measured choices: the x passes stay at 256 threads
// (with their batched row staging, 16 values per thread at n_x/2 = 420 beat
// 1024-thread workgroups by 10% forward, 4% inverse); the strided passes use
// at most 512 (1024 slowed them at 840; 16-line batches of 512 threads were 7%
// slower than 8 lines of 256 at 256^3).
int choose_lines(ins::FftPlan& pl, int maxl, int want, int wide, size_t extra, bool occ, int wide10 = 0) {
    struct Shape {
        int vm, nth;
    };
    const Shape shapes[4] = {{8, kBlockHost}, {8, wide}, {10, wide10}, {16, kBlockHost}};
    int best = -1;
    for (const Shape& sh : shapes) {
        if (sh.nth == 0) continue;
        const int lp = lines_for(pl, maxl, sh.vm, 1, sh.nth, extra);
        const int l0 = lines_for(pl, maxl, sh.vm, 0, sh.nth, extra);
        const int l = std::max(lp, l0);
        if (l <= best) continue;
        pl.vm = sh.vm;
        pl.nth = sh.nth;
        pl.pad = lp >= l0 && (!occ || kCuLds / fft_lds(pl, 1 << l, 1, extra) >= kCuLds / fft_lds(pl, 1 << l, 0, extra))
                     ? 1
                     : 0;
        best = l;
        if ((1 << l) >= want) break;
    }
    return best;
}

struct Pending {
    const char* name;
    hipEvent_t a, b;
};

// Fixed device scratch of the allocation-free entry point ins_stats_noalloc:
// the per-workgroup partials of the capped statistics kernel (4 doubles per
// workgroup, 64 KiB). Each device holds its own copy for the life of the
// process. Host code never names the array in a kernel argument or copy: it
// uses the device address looked up once per device (scratch_on).
constexpr size_t kScratchDoubles = 4 * size_t(ins::kStatsCapBlocks);
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`, looked up with
// hipGetSymbolAddress on the first call for that device (ins_create).
double* scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) raise(INS_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) raise(INS_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_dev[dev];
}

}  // namespace

struct ins_ctx_s {
    ins::Grid g{};
    ins_dtype dtype = INS_FP64;
    int device = 0;
    hipStream_t stream = nullptr;

    bool walls = false;  // no-slip walls at both y ends (INS_BC_WALLS_Y)
    // channel pressure solver: direct (x, z FFTs + tridiagonal solves along y,
    // when the sizes allow it) or conjugate gradients
    bool direct_ok = false;
    bool use_direct = false;
    double wy = 0.0;  // sum_j w_j (the channel height)

    // conjugate-gradient solve of the channel grid
    double cg_rtol = 1e-10;
    int cg_maxiter = 20000;
    int cg_check = 16;  // iterations between host convergence checks (0: never; all cg_maxiter launched)
    double* cg_r = nullptr;
    double* cg_p[2] = {nullptr, nullptr};
    double* cg_part = nullptr;  // partial sums: mean, rr and p.q (two generations each); cg_blocks * batch each
    ins::CgScal* cg_st = nullptr;
    ins::CgScal* cg_host = nullptr;  // pinned host copy of cg_st
    double* d_ym = nullptr;          // y metrics of the channel grid (Grid::ym)
    // stretched grid (a periodic direction, or the channel's x or z, given faces):
    // every operator from the per-direction metrics Grid::gm, pressure by CG
    bool gen = false;
    double* d_gm = nullptr;
    std::vector<double> faces[3];    // host copy of the faces given per direction (empty: uniform)
    double wsum = 0.0;               // sum of the cell volumes' y widths over one field (n_x n_z sum_j w_j)

    ins::FftPlan px{}, py{}, pz{};
    ins::FftPlan py_rev{}, pz_rev{};  // radices reversed: inverse half of the fused last-axis solve
    int lnl_x = 0, lnl_y = 0, lnl_z = 0;
    cd* d_tw = nullptr;
    cd* d_post = nullptr;
    double* d_lam = nullptr;
    // all-float32 comparison mode: float32 tables; spec then holds cf values
    ins::cf* d_twf = nullptr;
    ins::cf* d_postf = nullptr;
    float* d_lamf = nullptr;
    ins::SolveTab st{};

    cd* spec = nullptr;
    double* p = nullptr;
    void* ry = nullptr;
    void* wa = nullptr;
    void* wb = nullptr;
    double* partials = nullptr;
    int nstat = 0;
    double* scratch = nullptr;  // this device's address of the fixed scratch (ins_stats_noalloc)

    // reverse-pass stage storage (allocated on first use)
    void* w2 = nullptr;
    void* w3 = nullptr;
    void* w4 = nullptr;
    double* p2 = nullptr;
    double* p3 = nullptr;
    double* p4 = nullptr;

    // learned closure (allocated by ins_closure_set)
    bool clos_on = false;     // a closure term is part of the right-hand side
    int clos_kind = 0;        // 1: learned CNN, 2: Smagorinsky eddy viscosity
    bool clos_alloc = false;  // CNN workspace allocated
    bool clos_common = false; // stage / cotangent buffers shared by both kinds allocated
    double eddy_c2 = 0.0;     // (C_s Delta)^2
    void* eddy_nu = nullptr;  // eddy viscosity at the pressure points of the last closure_forward
    void* eddy_P = nullptr;   // pullback scratch
    const void* eddy_u = nullptr;  // velocity of the last closure_forward (read by its pullback)
    float* theta = nullptr;      // float32 parameters (device copy)
    float* theta_bar = nullptr;  // accumulated parameter gradient
    unsigned short* wf[3] = {nullptr, nullptr, nullptr};  // packed forward weights per layer
    unsigned short* wd[3] = {nullptr, nullptr, nullptr};  // packed dgrad weights per layer
    unsigned short *x0 = nullptr, *a1 = nullptr, *a2 = nullptr, *gm = nullptr, *gz1 = nullptr, *gz2 = nullptr;
    float *z1 = nullptr, *z2 = nullptr, *partial = nullptr;
    void* mclos = nullptr;  // closure term at the current stage (velocity layout)
    void* ui = nullptr;     // materialised stage velocity
    void* fbar = nullptr;   // right-hand-side cotangent of the current reverse stage

    size_t bytes = 0;
    std::vector<void*> allocs;

    bool prof = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<int64_t, double>> totals;
    std::vector<std::string> order;

    size_t vel_bytes() const {
        return static_cast<size_t>(g.batch) * g.dim * g.ncell * (dtype == INS_FP64 ? 8 : 4);
    }
    // pressure-point fields: float64, float32 in the all-float32 comparison mode
    size_t scal_bytes() const { return static_cast<size_t>(g.batch) * g.ncell * (dtype == INS_FP32_ALL ? 4 : 8); }
    bool f32all() const { return dtype == INS_FP32_ALL; }

    void* alloc(size_t n) {
        void* ptr = nullptr;
        if (hipMalloc(&ptr, n) != hipSuccess) {
            (void)hipGetLastError();
            raise(INS_ERR_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        allocs.push_back(ptr);
        bytes += n;
        return ptr;
    }

    hipEvent_t event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "hipEventCreate");
        return e;
    }

    template <class F>
    void launch(const char* name, F&& f) {
        hipEvent_t a = nullptr, b = nullptr;
        if (prof) {
            a = event();
            b = event();
            hip_check(hipEventRecord(a, stream), "hipEventRecord");
        }
        const hipError_t e = f();
        if (e != hipSuccess) raise(INS_ERR_HIP, std::string(name) + ": " + hipGetErrorString(e));
        if (prof) {
            hip_check(hipEventRecord(b, stream), "hipEventRecord");
            pending.push_back({name, a, b});
        }
    }

    void collect() {
        if (pending.empty()) return;
        hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
        for (auto& pr : pending) {
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, pr.a, pr.b), "hipEventElapsedTime");
            auto it = totals.find(pr.name);
            if (it == totals.end()) {
                totals[pr.name] = {1, ms};
                order.push_back(pr.name);
            } else {
                it->second.first += 1;
                it->second.second += ms;
            }
            pool.push_back(pr.a);
            pool.push_back(pr.b);
        }
        pending.clear();
    }

    ~ins_ctx_s() {
        for (auto& pr : pending) {
            (void)hipEventDestroy(pr.a);
            (void)hipEventDestroy(pr.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
        for (void* ptr : allocs) (void)hipFree(ptr);
        if (cg_host) (void)hipHostFree(cg_host);
    }
};

namespace {

template <class F>
ins_status guarded(F&& f) {
    try {
        f();
        return INS_OK;
    } catch (const InsError& e) {
        g_last_error = e.msg;
        return e.st;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return INS_ERR_INVALID;
    } catch (...) {
        g_last_error = "unknown error";
        return INS_ERR_INVALID;
    }
}

void need(const void* ptr, const char* what) {
    if (!ptr) raise(INS_ERR_INVALID, std::string(what) + " is null");
}

// Entry points that need float64 pressure-point fields (pullbacks through a
// solve, kept stages, closures, stretched grids, the energy spectrum): the
// all-float32 comparison mode covers the forward operators and steps only.
void no_f32all(ins_ctx c, const char* what) {
    if (c->dtype == INS_FP32_ALL)
        raise(INS_ERR_UNSUPPORTED, std::string(what) + " is not available in the all-float32 comparison mode");
}

void periodic_only(ins_ctx c, const char* what) {
    if (c->walls) raise(INS_ERR_UNSUPPORTED, std::string(what) + " needs the periodic grid");
    if (c->gen) raise(INS_ERR_UNSUPPORTED, std::string(what) + " needs the uniform periodic grid");
}

ins_ctx checked(ins_ctx c) {
    if (!c) raise(INS_ERR_INVALID, "context is null");
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != c->device) hip_check(hipSetDevice(c->device), "hipSetDevice");
    return c;
}

template <class F>
void with_type(ins_ctx c, F&& f) {
    if (c->dtype == INS_FP64)
        f(double{});
    else
        f(float{});
}

// y metrics of the channel (Grid::ym) from the cell widths (uniform: every
// width h_y, weights exactly 1/2) or from the face coordinates.
void upload_y_metrics(ins_ctx c, const double* faces) {
    ins::Grid& g = c->g;
    const int ny = g.ny, S = ny + 2;
    std::vector<double> w(ny), d(ny + 1), th(ny, 0.5);
    if (faces) {
        std::vector<double> cen(ny);
        for (int j = 0; j < ny; ++j) {
            w[j] = faces[j + 1] - faces[j];
            cen[j] = 0.5 * (faces[j] + faces[j + 1]);
        }
        d[0] = w[0];
        for (int j = 0; j + 1 < ny; ++j) {
            d[j + 1] = cen[j + 1] - cen[j];
            th[j] = w[j] / (w[j] + w[j + 1]);
        }
        d[ny] = w[ny - 1];
    } else {
        const double h = 1.0 / g.ih[1];
        std::fill(w.begin(), w.end(), h);
        std::fill(d.begin(), d.end(), h);
    }
    std::vector<double> m(5 * size_t(S), 0.0);
    double sw = 0.0;
    for (int j = 0; j < ny; ++j) {
        m[j] = 1.0 / w[j];
        m[2 * S + j] = th[j];
        m[3 * S + j] = w[j];
        sw += w[j];
    }
    for (int j = 0; j <= ny; ++j) {
        m[S + j] = 1.0 / d[j];
        m[4 * S + j] = d[j];
    }
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    hip_check(hipMemcpy(c->d_ym, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice), "upload y metrics");
    c->wsum = sw * double(g.nx) * double(g.nz);
    c->wy = sw;
    g.ym = c->d_ym;
}

// Stretched grid: per-direction metrics for i = -1 .. n (layout in Grid::gm):
// the faces given for that direction or the uniform spacing of the box;
// periodic images wrap, beyond the channel's walls the first / last row is
// mirrored (d_{-1} = w_0, d_{n-1} = w_{n-1}, theta = 1/2). wsum becomes the
// total volume (the CG's weighted means use the full cell volumes here).
void upload_gen_metrics(ins_ctx c) {
    ins::Grid& g = c->g;
    const int d = g.dim;
    const int n[3] = {g.nx, g.ny, g.nz};
    size_t total = 0;
    for (int a = 0; a < d; ++a) total += 5 * size_t(n[a] + 2);
    if (!c->d_gm) c->d_gm = static_cast<double*>(c->alloc(total * sizeof(double)));
    std::vector<double> m(total, 0.0);
    double vol = 1.0;
    size_t off = 0;
    for (int a = 0; a < d; ++a) {
        const int N = n[a], S = N + 2;
        std::vector<double> w(N);
        if (c->faces[a].empty()) {
            std::fill(w.begin(), w.end(), 1.0 / g.ih[a]);
        } else {
            for (int i = 0; i < N; ++i) w[i] = c->faces[a][i + 1] - c->faces[a][i];
        }
        const bool per = !(a == 1 && c->walls);
        auto W = [&](int i) { return per ? w[((i % N) + N) % N] : w[std::min(std::max(i, 0), N - 1)]; };
        double len = 0.0;
        for (int i = 0; i < N; ++i) len += w[i];
        for (int i = -1; i <= N; ++i) {
            const double wi = W(i);
            double di, thi;
            if (per || (i >= 0 && i <= N - 2)) {
                di = 0.5 * (W(i) + W(i + 1));
                thi = W(i) / (W(i) + W(i + 1));
            } else {
                di = W(i);
                thi = 0.5;
            }
            m[off + i + 1] = 1.0 / wi;
            m[off + S + i + 1] = 1.0 / di;
            m[off + 2 * S + i + 1] = thi;
            m[off + 3 * S + i + 1] = wi;
            m[off + 4 * S + i + 1] = di;
        }
        vol *= len;
        off += 5 * size_t(S);
    }
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    hip_check(hipMemcpy(c->d_gm, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice), "upload grid metrics");
    off = 0;
    for (int a = 0; a < d; ++a) {
        g.gm[a] = c->d_gm + off;
        off += 5 * size_t(n[a] + 2);
    }
    g.ywalls = c->walls ? 1 : 0;
    c->wsum = vol;
}

// Switch a context to the stretched-grid operators (irreversible): the CG
// workspace of the pressure solve is allocated here for a periodic context.
void enter_gen(ins_ctx c) {
    if (c->clos_on) raise(INS_ERR_UNSUPPORTED, "closures need the uniform periodic grid: clear the closure first");
    if (!c->cg_r) {
        const ins::Grid& g = c->g;
        const size_t sb = c->scal_bytes();
        c->cg_r = static_cast<double*>(c->alloc(sb));
        c->cg_p[0] = static_cast<double*>(c->alloc(sb));
        c->cg_p[1] = static_cast<double*>(c->alloc(sb));
        c->cg_part = static_cast<double*>(c->alloc(5 * size_t(ins::cg_blocks(g)) * g.batch * sizeof(double)));
        c->cg_st = static_cast<ins::CgScal*>(c->alloc(size_t(g.batch) * sizeof(ins::CgScal)));
        hip_check(hipMemset(c->cg_st, 0, size_t(g.batch) * sizeof(ins::CgScal)), "hipMemset");
        hip_check(hipHostMalloc(reinterpret_cast<void**>(&c->cg_host), size_t(g.batch) * sizeof(ins::CgScal)),
                  "hipHostMalloc");
    }
    c->use_direct = false;
    c->direct_ok = false;
    c->gen = true;
}

bool cg_all_done(ins_ctx c) {
    const size_t nb = size_t(c->g.batch) * sizeof(ins::CgScal);
    hip_check(hipMemcpyAsync(c->cg_host, c->cg_st, nb, hipMemcpyDeviceToHost, c->stream), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    for (int b = 0; b < c->g.batch; ++b)
        if (!c->cg_host[b].done) return false;
    return true;
}

// Channel grid: x = (D G)^+ of the divergence of vel or of r, by conjugate
// gradients on -D G (Sec. 2.6.1, iterative solver) from x = 0; the mean of
// the right-hand side is removed first (the zero-mean solution of the
// consistent part). Iterations are launched back to back; every cg_check
// iterations the host reads the stop flags once and stops launching when
// every field is done.
// mode 0: x = L^+ D vel; 1: x = L^+ D Omega_u^{-1} vel (inside the transposed
// projection Omega_u P Omega_u^{-1}); 2: x = L^+ r; 3: the inner solve of the
// pullback of 2 (right-hand side mean(r) - r unscaled, see ins_poisson_solve_vjp).
// The operator is the symmetric -Omega_p D G, the right-hand side of modes
// 0-2 is Omega_p (mean_w - r) with mean_w the volume-weighted mean.
void cg_solve(ins_ctx c, const void* vel, const double* r, double* x, int mode) {
    const ins::Grid& g = c->g;
    const size_t np = size_t(ins::cg_blocks(g)) * g.batch;
    double* msum = c->cg_part;
    double* rb[2] = {c->cg_part + np, c->cg_part + 2 * np};
    double* pq[2] = {c->cg_part + 3 * np, c->cg_part + 4 * np};
    if (vel) {
        with_type(c, [&](auto tag) {
            using T = decltype(tag);
            c->launch("cg_div", [&] {
                return ins::launch_cg_div<T>(g, static_cast<const T*>(vel), nullptr, c->cg_r, msum, mode, c->stream);
            });
        });
    } else {
        c->launch("cg_copy", [&] { return ins::launch_cg_div<double>(g, nullptr, r, c->cg_r, msum, mode, c->stream); });
    }
    c->launch("cg_init", [&] {
        return ins::launch_cg_init(g, c->cg_r, x, msum, rb[0], c->cg_st, mode, c->wsum, c->stream);
    });
    const double rtol2 = c->cg_rtol * c->cg_rtol;
    auto apply = [&](int k) {
        c->launch("cg_apply", [&] {
            return ins::launch_cg_apply(g, c->cg_r, c->cg_p[k & 1], c->cg_p[(k + 1) & 1], x, rb[k & 1],
                                        rb[(k + 1) & 1], pq[(k + 1) & 1], pq[k & 1], c->cg_st, k, rtol2, c->cg_maxiter,
                                        c->stream);
        });
    };
    int k = 0;
    while (k < c->cg_maxiter) {
        apply(k);
        c->launch("cg_update", [&] {
            return ins::launch_cg_update(g, c->cg_r, c->cg_p[(k + 1) & 1], rb[k & 1], pq[k & 1], rb[(k + 1) & 1],
                                         c->cg_st, k, rtol2, c->cg_maxiter, c->stream);
        });
        ++k;
        if (c->cg_check > 0 && k % c->cg_check == 0 && k < c->cg_maxiter && cg_all_done(c)) break;
    }
    // every field is stopped at k: this launch only applies the last pending x update
    apply(k);
    c->launch("cg_finish", [&] { return ins::launch_cg_finish(g, rb[k & 1], c->cg_st, c->stream); });
}

// Channel grid, direct solve: x = the zero-mean solution of D G x = r' with r'
// = r - mean_w(r), r the divergence of vel or given. Modes as for cg_solve
// (0: D vel, 1: D Omega_u^{-1} vel, 2: r, 3: the transpose of mode 2's map).
// Forward FFTs along x (fused with the divergence) and z, one tridiagonal
// solve along y per wavenumber pair, inverse FFTs.
void direct_solve(ins_ctx c, const void* vel, const double* r, double* x, int mode) {
    const ins::Grid& g = c->g;
    if (vel) {
        with_type(c, [&](auto tag) {
            using T = decltype(tag);
            c->launch("fft_x_fwd_div", [&] {
                return ins::launch_fft_x_fwd_wall<T>(g, static_cast<const T*>(vel), mode == 1, c->spec, c->px,
                                                     c->d_post, c->lnl_x, c->stream);
            });
        });
    } else {
        c->launch("fft_x_fwd", [&] {
            return ins::launch_fft_x_fwd<double>(g, nullptr, r, c->spec, c->px, c->d_post, c->lnl_x, c->stream);
        });
    }
    if (g.dim == 3)
        c->launch("fft_z_fwd", [&] { return ins::launch_fft_strided(g, c->spec, c->pz, c->pz, 2, 0, c->lnl_z, c->st, c->stream); });
    const double scale = 1.0 / (double(g.nx) * double(g.nz));
    c->launch("channel_ysolve", [&] {
        return ins::launch_channel_ysolve(g, c->spec, c->st.lam[0], c->st.lam[2], c->wy, scale, mode == 3, c->stream);
    });
    if (g.dim == 3)
        c->launch("fft_z_inv", [&] { return ins::launch_fft_strided(g, c->spec, c->pz, c->pz, 2, 1, c->lnl_z, c->st, c->stream); });
    c->launch("fft_x_inv", [&] { return ins::launch_fft_x_inv(g, c->spec, x, c->px, c->d_post, c->lnl_x, c->stream); });
}

// p = (D G)^-1 of the divergence of vel (vel != null) or of r. adj (channel):
// the solve inside the transposed projection, of D Omega_u^{-1} vel.
// All-float32 comparison mode: the spectral solve of poisson() on a float32
// spectrum; r and p hold float32 values.
void poisson_f32(ins_ctx c, const void* vel, const float* r, float* p) {
    const ins::Grid& g = c->g;
    ins::cf* spec = reinterpret_cast<ins::cf*>(c->spec);
    c->launch(vel ? "fft_x_fwd_div" : "fft_x_fwd", [&] {
        return ins::launch_fft_x_fwd_f32(g, static_cast<const float*>(vel), r, spec, c->px, c->d_postf, c->lnl_x,
                                         c->stream);
    });
    if (g.dim == 3) {
        c->launch("fft_y_fwd", [&] { return ins::launch_fft_strided_f32(g, spec, c->py, c->py, 1, 0, c->lnl_y, c->st, c->stream); });
        c->launch("fft_z_solve", [&] { return ins::launch_fft_strided_f32(g, spec, c->pz, c->pz_rev, 2, 2, c->lnl_z, c->st, c->stream); });
        c->launch("fft_y_inv", [&] { return ins::launch_fft_strided_f32(g, spec, c->py, c->py, 1, 1, c->lnl_y, c->st, c->stream); });
    } else {
        c->launch("fft_y_solve", [&] { return ins::launch_fft_strided_f32(g, spec, c->py, c->py_rev, 1, 2, c->lnl_y, c->st, c->stream); });
    }
    c->launch("fft_x_inv", [&] { return ins::launch_fft_x_inv_f32(g, spec, p, c->px, c->d_postf, c->lnl_x, c->stream); });
}

void poisson(ins_ctx c, const void* vel, const double* r, double* p, bool adj = false) {
    const ins::Grid& g = c->g;
    if (c->f32all()) {
        // pressure-point buffers hold float32 values in this mode
        poisson_f32(c, vel, reinterpret_cast<const float*>(r), reinterpret_cast<float*>(p));
        return;
    }
    if (c->walls || c->gen) {
        if (c->use_direct)
            direct_solve(c, vel, r, p, vel ? (adj ? 1 : 0) : 2);
        else
            cg_solve(c, vel, r, p, vel ? (adj ? 1 : 0) : 2);
        return;
    }
    if (vel) {
        with_type(c, [&](auto tag) {
            using T = decltype(tag);
            c->launch("fft_x_fwd_div", [&] {
                return ins::launch_fft_x_fwd<T>(g, static_cast<const T*>(vel), nullptr, c->spec, c->px, c->d_post,
                                                c->lnl_x, c->stream);
            });
        });
    } else {
        c->launch("fft_x_fwd", [&] {
            return ins::launch_fft_x_fwd<double>(g, nullptr, r, c->spec, c->px, c->d_post, c->lnl_x, c->stream);
        });
    }
    if (g.dim == 3) {
        c->launch("fft_y_fwd", [&] { return ins::launch_fft_strided(g, c->spec, c->py, c->py, 1, 0, c->lnl_y, c->st, c->stream); });
        c->launch("fft_z_solve", [&] { return ins::launch_fft_strided(g, c->spec, c->pz, c->pz_rev, 2, 2, c->lnl_z, c->st, c->stream); });
        c->launch("fft_y_inv", [&] { return ins::launch_fft_strided(g, c->spec, c->py, c->py, 1, 1, c->lnl_y, c->st, c->stream); });
    } else {
        c->launch("fft_y_solve", [&] { return ins::launch_fft_strided(g, c->spec, c->py, c->py_rev, 1, 2, c->lnl_y, c->st, c->stream); });
    }
    c->launch("fft_x_inv", [&] { return ins::launch_fft_x_inv(g, c->spec, p, c->px, c->d_post, c->lnl_x, c->stream); });
}


// out = w - G p; adj (channel): w - Omega_u G p, completing the transposed
// projection Omega_u P Omega_u^{-1} (on the periodic grid P^T = P).
template <typename T>
void apply_projection(ins_ctx c, const T* w, const double* p, T* out, bool adj = false) {
    if (c->f32all()) {
        c->launch("apply_projection", [&] {
            return ins::launch_apply_projection_f32(c->g, reinterpret_cast<const float*>(w),
                                                    reinterpret_cast<const float*>(p), reinterpret_cast<float*>(out),
                                                    c->stream);
        });
        return;
    }
    if (c->gen) {
        c->launch("gen_projection", [&] { return ins::launch_gen_project<T>(c->g, w, p, out, adj, c->stream); });
        return;
    }
    if (c->walls) {
        c->launch("wall_projection", [&] { return ins::launch_wall_project<T>(c->g, w, p, out, adj, c->stream); });
        return;
    }
    c->launch("apply_projection", [&] { return ins::launch_apply_projection<T>(c->g, w, p, out, c->stream); });
}

// ----------------------------------------------------------------------------
// Learned closure m_theta (Sec. 4): parameter layout per layer W[out][in][kz][ky][kx]
// then b[out], layers (3->32), (32->32), (32->3).
// ----------------------------------------------------------------------------
constexpr int kClosParams = 32899;
constexpr int kW1 = 0, kB1 = 2592, kW2 = 2624, kB2 = 30272, kW3 = 30304, kB3 = 32896;

void closure_alloc_common(ins_ctx c) {
    if (c->clos_common) return;
    c->mclos = c->alloc(c->vel_bytes());
    c->ui = c->alloc(c->vel_bytes());
    c->fbar = c->alloc(c->vel_bytes());
    c->clos_common = true;
}

void closure_alloc(ins_ctx c) {
    if (c->clos_alloc) return;
    const size_t n = size_t(c->g.ncell) * c->g.batch;
    c->theta = static_cast<float*>(c->alloc(kClosParams * sizeof(float)));
    c->theta_bar = static_cast<float*>(c->alloc(kClosParams * sizeof(float)));
    // packed sizes: forward NKT(cinp) * ntf * 512, dgrad NKT(coutp) * ntd * 512 (bf16 words)
    const size_t wf_sz[3] = {7 * 2 * 512, 27 * 2 * 512, 27 * 1 * 512};
    const size_t wd_sz[3] = {27 * 1 * 512, 27 * 2 * 512, 7 * 2 * 512};
    for (int l = 0; l < 3; ++l) {
        c->wf[l] = static_cast<unsigned short*>(c->alloc(wf_sz[l] * 2));
        c->wd[l] = static_cast<unsigned short*>(c->alloc(wd_sz[l] * 2));
    }
    c->x0 = static_cast<unsigned short*>(c->alloc(n * 8 * 2));
    c->gm = static_cast<unsigned short*>(c->alloc(n * 8 * 2));
    c->a1 = static_cast<unsigned short*>(c->alloc(n * 32 * 2));
    c->a2 = static_cast<unsigned short*>(c->alloc(n * 32 * 2));
    c->gz1 = static_cast<unsigned short*>(c->alloc(n * 32 * 2));
    c->gz2 = static_cast<unsigned short*>(c->alloc(n * 32 * 2));
    c->z1 = static_cast<float*>(c->alloc(n * 32 * 4));
    c->z2 = static_cast<float*>(c->alloc(n * 32 * 4));
    c->partial = static_cast<float*>(c->alloc(ins::closure_wgrad_partial_floats(int64_t(n)) * 4));
    closure_alloc_common(c);
    c->clos_alloc = true;
    c->launch("fill_zero", [&] { return ins::launch_fill_zero_f(c->theta_bar, kClosParams, c->stream); });
}

void eddy_alloc(ins_ctx c) {
    if (c->eddy_nu) return;
    const size_t es = c->dtype == INS_FP64 ? 8 : 4;
    const size_t n = size_t(c->g.ncell) * c->g.batch;
    const int d = c->g.dim;
    c->eddy_nu = c->alloc(n * es);
    c->eddy_P = c->alloc(n * es * size_t(d * (d + 1) / 2));
    closure_alloc_common(c);
}

// m = m_theta(u); leaves x0, z1, a1, z2, a2 for a following pullback.
template <typename T>
void closure_forward(ins_ctx c, const T* u, T* m, bool keep_z = true) {
    const ins::Grid& g = c->g;
    if (c->clos_kind == 2) {
        c->eddy_u = u;
        c->launch("eddy_forward", [&] {
            return ins::launch_eddy_forward<T>(g, u, static_cast<T*>(c->eddy_nu), m, c->eddy_c2, c->stream);
        });
        return;
    }
    // the float32 pre-activations are kept only when a pullback will need them
    float* z1 = keep_z ? c->z1 : nullptr;
    float* z2 = keep_z ? c->z2 : nullptr;
    c->launch("cnn_pack_input", [&] { return ins::launch_closure_pack_input<T>(g, u, c->x0, c->stream); });
    c->launch("cnn_conv1", [&] {
        return ins::launch_closure_conv<T>(g, 0, c->x0, c->wf[0], c->theta + kB1, nullptr, z1, c->a1, nullptr, c->stream);
    });
    c->launch("cnn_conv2", [&] {
        return ins::launch_closure_conv<T>(g, 1, c->a1, c->wf[1], c->theta + kB2, nullptr, z2, c->a2, nullptr, c->stream);
    });
    c->launch("cnn_conv3", [&] {
        return ins::launch_closure_conv<T>(g, 2, c->a2, c->wf[2], c->theta + kB3, nullptr, nullptr, nullptr, m, c->stream);
    });
}

// ubar += (d m / d u)^T mbar and theta_bar += (d m / d theta)^T mbar, at the u of
// the last closure_forward.
template <typename T>
void closure_backward(ins_ctx c, const T* mbar, T* ubar) {
    const ins::Grid& g = c->g;
    if (c->clos_kind == 2) {
        // at the u of the last closure_forward (the stage velocity, or the caller's u)
        c->launch("eddy_backward", [&] {
            return ins::launch_eddy_backward<T>(g, static_cast<const T*>(c->eddy_u), static_cast<const T*>(c->eddy_nu), mbar,
                                                static_cast<T*>(c->eddy_P), ubar, c->eddy_c2, c->stream);
        });
        return;
    }
    c->launch("cnn_pack_cotangent", [&] { return ins::launch_closure_pack_input<T>(g, mbar, c->gm, c->stream); });
    c->launch("cnn_dgrad3", [&] {
        return ins::launch_closure_conv<T>(g, 10, c->gm, c->wd[2], nullptr, c->z2, nullptr, c->gz2, nullptr, c->stream);
    });
    c->launch("cnn_wgrad3", [&] {
        return ins::launch_closure_wgrad(g, 2, c->gm, c->a2, c->partial, c->theta_bar + kW3, c->theta_bar + kB3, c->stream);
    });
    c->launch("cnn_dgrad2", [&] {
        return ins::launch_closure_conv<T>(g, 11, c->gz2, c->wd[1], nullptr, c->z1, nullptr, c->gz1, nullptr, c->stream);
    });
    c->launch("cnn_wgrad2", [&] {
        return ins::launch_closure_wgrad(g, 1, c->gz2, c->a1, c->partial, c->theta_bar + kW2, c->theta_bar + kB2, c->stream);
    });
    c->launch("cnn_dgrad1", [&] {
        return ins::launch_closure_conv<T>(g, 12, c->gz1, c->wd[0], nullptr, nullptr, nullptr, nullptr, ubar, c->stream);
    });
    c->launch("cnn_wgrad1", [&] {
        return ins::launch_closure_wgrad(g, 0, c->gz1, c->x0, c->partial, c->theta_bar + kW1, c->theta_bar + kB1, c->stream);
    });
}

// Closure term at the stage velocity u_i = (p ? w - G p : w); returns m or nullptr.
template <typename T>
const T* closure_at_stage(ins_ctx c, const T* w, const double* p, bool keep_z = false) {
    if (!c->clos_on) return nullptr;
    const T* u = w;
    if (p) {
        T* ui = static_cast<T*>(c->ui);
        apply_projection<T>(c, w, p, ui);
        u = ui;
    }
    T* m = static_cast<T*>(c->mclos);
    closure_forward<T>(c, u, m, keep_z);
    return m;
}

template <typename T>
// ymode: 0 reads the accumulator y, 1 starts it at u0, 2 forms it as
// u0 + (wprev - u0)/3 + 2 (w - u0)/3 from the unprojected stage inputs (RK4's
// third stage, periodic 3D only; wprev may be wout's buffer).
void stage(ins_ctx c, const T* w, const double* p, bool proj, const T* u0, T* y, int ymode, double cy, T* wout,
           double cw, const char* label = nullptr, const T* wprev = nullptr) {
    const bool yinit = ymode == 1;
    // one profile name per data-movement variant (their byte counts differ)
    const char* name = label ? label
                             : !proj ? (y ? "stage_first" : "stage_first_rec")
                                     : (y ? (wout ? (ymode == 2 ? "stage_yw" : "stage") : "stage_last") : "stage_rec");
    if (ymode == 2) {
        if (c->f32all() || c->gen || c->walls || c->g.dim != 3 || !proj || !y || !wout || !wprev)
            raise(INS_ERR_UNSUPPORTED, "accumulator from the stage inputs: periodic 3D projected stages only");
        const T* mc = closure_at_stage<T>(c, w, p);
        c->launch(name, [&] {
            return ins::launch_stage_zm_yw<T>(c->g, w, p, u0, wprev, 1.0 / 3.0, 2.0 / 3.0, y, cy, wout, cw, c->stream,
                                              mc);
        });
        return;
    }
    if (c->f32all()) {
        c->launch(name, [&] {
            return ins::launch_stage_f32(c->g, reinterpret_cast<const float*>(w), reinterpret_cast<const float*>(p),
                                         proj, reinterpret_cast<const float*>(u0), reinterpret_cast<float*>(y), yinit,
                                         cy, reinterpret_cast<float*>(wout), cw, c->stream);
        });
        return;
    }
    if (c->gen) {
        c->launch(name, [&] { return ins::launch_gen_stage<T>(c->g, w, p, proj, u0, y, yinit, cy, wout, cw, c->stream); });
        return;
    }
    if (c->walls) {
        c->launch(name, [&] { return ins::launch_wall_stage<T>(c->g, w, p, proj, u0, y, yinit, cy, wout, cw, c->stream); });
        return;
    }
    const T* mc = closure_at_stage<T>(c, w, proj ? p : nullptr);
    c->launch(name, [&] {
        return ins::launch_stage<T>(c->g, w, p, proj, u0, y, yinit, cy, wout, cw, c->stream, mc);
    });
}

// Stage inputs of one step kept for its pullback: the unprojected stage sums
// W_i (velocity fields) and their pressures P_i (u_i = W_i - G P_i), i = 2..4
// for RK4 and 2..3 for Wray3. Either the context's reverse-pass storage or
// caller buffers (ins_step_save / ins_step_vjp_saved).
template <typename T>
struct Stages {
    T* w[3];
    double* p[3];
};

template <typename T>
Stages<T> own_stages(ins_ctx c) {
    return {{static_cast<T*>(c->w2), static_cast<T*>(c->w3), static_cast<T*>(c->w4)}, {c->p2, c->p3, c->p4}};
}

// Classical RK4, projection after every stage (Sec. 2.6.2), low-storage
// schedule: accumulator y, stage registers wa/wb, one pressure per stage.
// With `keep` the stage registers and pressures are the given buffers (the
// same work, their contents left for the pullback).
template <typename T>
void step_rk4(ins_ctx c, const T* u0, T* u1, double dt, const Stages<T>* keep = nullptr) {
    T* y = static_cast<T*>(c->ry);
    T* wa = static_cast<T*>(c->wa);
    T* wb = static_cast<T*>(c->wb);
    double* p = c->p;
    T* W2 = keep ? keep->w[0] : wa;
    T* W3 = keep ? keep->w[1] : wb;
    T* W4 = keep ? keep->w[2] : wa;
    double* P2 = keep ? keep->p[0] : p;
    double* P3 = keep ? keep->p[1] : p;
    double* P4 = keep ? keep->p[2] : p;
    // On the periodic 3D grid the first two stages store only W2 = u0 + dt/2 F1
    // and W3 = u0 + dt/2 F2: the third forms the accumulator
    // u0 + dt/6 F1 + dt/3 F2 = u0 + (W2 - u0)/3 + 2 (W3 - u0)/3 from W2 (read
    // pointwise before W4 overwrites it) and the u0 and W3 it reads anyway
    // (72 bytes per cell less traffic per step in float64).
    const bool yw = !c->f32all() && !c->gen && !c->walls && c->g.dim == 3;
    stage<T>(c, u0, nullptr, false, u0, yw ? nullptr : y, 1, dt / 6.0, W2, dt / 2.0);
    poisson(c, W2, nullptr, P2);
    stage<T>(c, W2, P2, true, u0, yw ? nullptr : y, 0, dt / 3.0, W3, dt / 2.0);
    poisson(c, W3, nullptr, P3);
    stage<T>(c, W3, P3, true, u0, y, yw ? 2 : 0, dt / 3.0, W4, dt, nullptr, yw ? W2 : nullptr);
    poisson(c, W4, nullptr, P4);
    stage<T>(c, W4, P4, true, u0, y, false, dt / 6.0, nullptr, 0.0);
    poisson(c, y, nullptr, p);
    apply_projection<T>(c, y, p, u1);
}

void ensure_vjp_storage(ins_ctx c) {
    if (c->w2) return;
    c->w2 = c->alloc(c->vel_bytes());
    c->w3 = c->alloc(c->vel_bytes());
    c->w4 = c->alloc(c->vel_bytes());
    c->p2 = static_cast<double*>(c->alloc(c->scal_bytes()));
    c->p3 = static_cast<double*>(c->alloc(c->scal_bytes()));
    c->p4 = static_cast<double*>(c->alloc(c->scal_bytes()));
}

template <typename T>
void stage_vjp(ins_ctx c, const T* w, const double* p, bool proj_u, const T* ybar, const T* un, const double* q,
               bool has_w, double cb, double cw, T* u0bar, int mode, T* out) {
    const char* name = mode == 0 ? "stage_vjp_first" : (mode >= 2 ? "stage_vjp_last" : "stage_vjp");
    if (c->gen) {
        c->launch(name, [&] {
            return ins::launch_gen_stage_vjp<T>(c->g, w, p, proj_u, ybar, un, q, has_w, cb, cw, u0bar, mode, out,
                                                c->stream);
        });
        return;
    }
    if (c->walls) {
        c->launch(name, [&] {
            return ins::launch_wall_stage_vjp<T>(c->g, w, p, proj_u, ybar, un, q, has_w, cb, cw, u0bar, mode, out,
                                                 c->stream);
        });
        return;
    }
    T* fb = c->clos_on ? static_cast<T*>(c->fbar) : nullptr;
    c->launch(name, [&] {
        return ins::launch_stage_vjp<T>(c->g, w, p, proj_u, ybar, un, q, has_w, cb, cw, u0bar, mode, out, c->stream, fb);
    });
    if (c->clos_on) {
        // the closure's share of the stage pullback: m_bar = Fbar_i, at u_i
        closure_at_stage<T>(c, w, proj_u ? p : nullptr, true);
        closure_backward<T>(c, fb, mode >= 2 ? u0bar : out);
    }
}

// Reverse pass of step_rk4 (Sec. 3.4) from the stage inputs S: project the
// incoming cotangent, then run the stages backwards. With ybar = P u1bar and
// wbar_{i+1} the projected cotangent of stage i+1's input:
//   Fbar_i = dt b_i ybar + dt a_{i+1} wbar_{i+1},  ubar_i = J_F(u_i)^T Fbar_i,
//   wbar_i = P ubar_i,  u0bar = ybar + sum_i wbar_i + ubar_1.
template <typename T>
void step_rk4_reverse(ins_ctx c, const T* u0, const Stages<T>& S, const T* u1bar, T* u0bar, double dt) {
    T* YB = static_cast<T*>(c->ry);
    T* UA = static_cast<T*>(c->wa);
    T* UB = static_cast<T*>(c->wb);
    double* Q = c->p;
    poisson(c, u1bar, nullptr, Q, true);
    apply_projection<T>(c, u1bar, Q, YB, true);
    stage_vjp<T>(c, S.w[2], S.p[2], true, YB, nullptr, nullptr, false, dt / 6.0, 0.0, u0bar, 0, UA);
    poisson(c, UA, nullptr, Q, true);
    stage_vjp<T>(c, S.w[1], S.p[1], true, YB, UA, Q, true, dt / 3.0, dt, u0bar, 1, UB);
    poisson(c, UB, nullptr, Q, true);
    stage_vjp<T>(c, S.w[0], S.p[0], true, YB, UB, Q, true, dt / 3.0, dt / 2.0, u0bar, 1, UA);
    poisson(c, UA, nullptr, Q, true);
    stage_vjp<T>(c, u0, nullptr, false, YB, UA, Q, true, dt / 6.0, dt / 2.0, u0bar, 2, nullptr);
}

// Pullback of step_rk4 that first recomputes the stage inputs from u0.
template <typename T>
void step_rk4_vjp(ins_ctx c, const T* u0, const T* u1bar, T* u0bar, double dt) {
    ensure_vjp_storage(c);
    const Stages<T> S = own_stages<T>(c);
    stage<T>(c, u0, nullptr, false, u0, nullptr, false, 0.0, S.w[0], dt / 2.0);
    poisson(c, S.w[0], nullptr, S.p[0]);
    stage<T>(c, S.w[0], S.p[0], true, u0, nullptr, false, 0.0, S.w[1], dt / 2.0);
    poisson(c, S.w[1], nullptr, S.p[1]);
    stage<T>(c, S.w[1], S.p[1], true, u0, nullptr, false, 0.0, S.w[2], dt);
    poisson(c, S.w[2], nullptr, S.p[2]);
    step_rk4_reverse<T>(c, u0, S, u1bar, u0bar, dt);
}

// Wray's low-storage three-stage scheme (Sec. 2.6.2 names it among the
// integrators, Sec. 3.3 as the low-storage one), projection after every
// stage. In Butcher form its stages are u_2 = P(u0 + dt 8/15 F_1),
// u_3 = P(u0 + dt (1/4 F_1 + 5/12 F_2)), u_new = P(u0 + dt (1/4 F_1 + 3/4 F_3));
// since both later sums start from yacc = u0 + dt/4 F_1, the schedule keeps
// yacc and one stage register: three stage kernels and three solves. With
// `keep`, W_2, W_3 and their pressures go to the given buffers.
template <typename T>
void step_wray3(ins_ctx c, const T* u0, T* u1, double dt, const Stages<T>* keep = nullptr) {
    T* yacc = static_cast<T*>(c->ry);
    T* wa = static_cast<T*>(c->wa);
    T* wb = static_cast<T*>(c->wb);
    double* p = c->p;
    T* W2 = keep ? keep->w[0] : wa;
    T* W3 = keep ? keep->w[1] : wb;
    double* P2 = keep ? keep->p[0] : p;
    double* P3 = keep ? keep->p[1] : p;
    stage<T>(c, u0, nullptr, false, u0, yacc, true, dt / 4.0, W2, dt * 8.0 / 15.0, "wray_stage1");
    poisson(c, W2, nullptr, P2);
    stage<T>(c, W2, P2, true, yacc, nullptr, false, 0.0, W3, dt * 5.0 / 12.0, "wray_stage2");
    poisson(c, W3, nullptr, P3);
    stage<T>(c, W3, P3, true, yacc, nullptr, false, 0.0, wa, dt * 3.0 / 4.0, "wray_stage3");
    poisson(c, wa, nullptr, p);
    apply_projection<T>(c, wa, p, u1);
}

// Reverse pass of step_wray3 from the stage inputs S. With w_2 = u0 + dt 8/15 F_1,
// yacc = u0 + dt/4 F_1, w_3 = yacc + dt 5/12 F_2(u_2), w_4 = yacc + dt 3/4 F_3(u_3), u_k = P w_k:
//   wbar_4 = P u1bar = yaccbar (so far); ubar_3 = J_F(u_3)^T (dt 3/4 wbar_4)
//   wbar_3 = P ubar_3; yaccbar += wbar_3; ubar_2 = J_F(u_2)^T (dt 5/12 wbar_3)
//   wbar_2 = P ubar_2; u0bar = yaccbar + wbar_2 + J_F(u0)^T (dt/4 yaccbar + dt 8/15 wbar_2).
template <typename T>
void step_wray3_reverse(ins_ctx c, const T* u0, const Stages<T>& S, const T* u1bar, T* u0bar, double dt) {
    T* YB = static_cast<T*>(c->ry);
    T* UA = static_cast<T*>(c->wa);
    T* UB = static_cast<T*>(c->wb);
    double* Q = c->p;
    poisson(c, u1bar, nullptr, Q, true);
    apply_projection<T>(c, u1bar, Q, YB, true);  // YB = wbar_4, the running yaccbar
    // the accumulator starts as YB itself, so this stage writes no accumulator
    stage_vjp<T>(c, S.w[1], S.p[1], true, YB, nullptr, nullptr, false, dt * 3.0 / 4.0, 0.0, nullptr, 0, UA);
    poisson(c, UA, nullptr, Q, true);
    // Fbar_2 = dt 5/12 wbar_3 (cb = 0, so the ybar operand is not YB, which this kernel updates)
    stage_vjp<T>(c, S.w[0], S.p[0], true, UA, UA, Q, true, 0.0, dt * 5.0 / 12.0, YB, 1, UB);
    poisson(c, UB, nullptr, Q, true);
    stage_vjp<T>(c, u0, nullptr, false, YB, UB, Q, true, dt / 4.0, dt * 8.0 / 15.0, u0bar, 3, nullptr);
}

// Pullback of step_wray3 that first recomputes W_2, W_3 (yacc passes through YB).
template <typename T>
void step_wray3_vjp(ins_ctx c, const T* u0, const T* u1bar, T* u0bar, double dt) {
    ensure_vjp_storage(c);
    const Stages<T> S = own_stages<T>(c);
    T* YB = static_cast<T*>(c->ry);
    stage<T>(c, u0, nullptr, false, u0, YB, true, dt / 4.0, S.w[0], dt * 8.0 / 15.0, "wray_stage1");
    poisson(c, S.w[0], nullptr, S.p[0]);
    stage<T>(c, S.w[0], S.p[0], true, YB, nullptr, false, 0.0, S.w[1], dt * 5.0 / 12.0, "wray_stage2");
    poisson(c, S.w[1], nullptr, S.p[1]);
    step_wray3_reverse<T>(c, u0, S, u1bar, u0bar, dt);
}

void check_dt(double dt) {
    if (!(dt > 0.0) || !std::isfinite(dt)) raise(INS_ERR_INVALID, "dt must be positive and finite");
}

}  // namespace

extern "C" {

const char* ins_last_error(void) { return g_last_error.c_str(); }

// FFT plans (x works on n_x/2 complex points), twiddles, the x untangling
// factors and the per-direction eigenvalues 4 sin^2(pi k / n) / h^2. Periodic
// grid: x, y, z passes and the fused solve along the last axis (its inverse
// runs the radices reversed). Channel: x and z passes only; returns false when
// a length does not fit a workgroup (the periodic grid raises instead).
bool setup_fft(ins_ctx c, const std::vector<int>& rx, const std::vector<int>& ry, const std::vector<int>& rz,
               bool channel) {
    ins::Grid& g = c->g;
    const int d = g.dim;
    std::vector<cd> tw;
    build_twiddles(g.nx / 2, rx, tw, c->px);
    if (!channel) build_twiddles(g.ny, ry, tw, c->py);
    if (d == 3) build_twiddles(g.nz, rz, tw, c->pz);
    // LDS beside the lines: the strided passes keep the roots (n/2 for even n, else n)
    // and, in the pass that divides by the eigenvalues, those of its axis
    auto strided_extra = [](int n, bool solve) {
        return static_cast<size_t>((n & 1) ? n : n / 2) * sizeof(cd) + (solve ? n * sizeof(double) : 0);
    };
    c->lnl_x = choose_lines(c->px, 16, 8, kBlockHost, 0, false, 512);
    c->lnl_y = channel ? 0 : choose_lines(c->py, 16, 8, 512, strided_extra(g.ny, d == 2), true);
    // the channel's z passes are plain forward / inverse transforms: 16-line batches
    // (256-byte runs) measured 13% faster there; the periodic fused z solve and the y
    // passes are faster with 8 lines of 256 threads
    c->lnl_z = d == 3 ? choose_lines(c->pz, 16, channel ? 16 : 8, 512, strided_extra(g.nz, !channel), true) : 0;
    if (!channel) {
        ins::FftPlan& last = d == 3 ? c->pz : c->py;
        ins::FftPlan& rev = d == 3 ? c->pz_rev : c->py_rev;
        std::vector<int> rr(d == 3 ? rz : ry);
        std::reverse(rr.begin(), rr.end());
        build_twiddles(last.n, rr, tw, rev);
        rev.vm = last.vm;
        rev.pad = last.pad;
        rev.nth = last.nth;
    }
    if (c->lnl_x < 0 || c->lnl_y < 0 || c->lnl_z < 0) {
        if (channel) return false;
        raise(INS_ERR_UNSUPPORTED, "FFT length too long");
    }

    const long double two_pi = 6.283185307179586476925286766559005768L;
    std::vector<cd> post(g.nx / 2 + 1);
    for (int k = 0; k <= g.nx / 2; ++k) {
        const long double ang = -two_pi * k / static_cast<long double>(g.nx);
        post[k] = cd{double(cosl(ang)), double(sinl(ang))};
    }
    // 4 sin^2(pi k / n) / h^2 per direction (Sec. 2.6.1 transfer function);
    // the channel's y entries are unused.
    std::vector<double> lam;
    size_t off[3] = {0, 0, 0};
    const int cnt[3] = {g.nx / 2 + 1, g.ny, d == 3 ? g.nz : 1};
    const int nn[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        off[a] = lam.size();
        for (int k = 0; k < cnt[a]; ++k) {
            if (a >= d) {
                lam.push_back(0.0);
                continue;
            }
            const long double s = sinl(two_pi * 0.5L * k / static_cast<long double>(nn[a]));
            lam.push_back(double(4.0L * s * s * static_cast<long double>(g.ih2[a])));
        }
    }
    c->d_tw = static_cast<cd*>(c->alloc(std::max<size_t>(tw.size(), 1) * sizeof(cd)));
    c->d_post = static_cast<cd*>(c->alloc(post.size() * sizeof(cd)));
    c->d_lam = static_cast<double*>(c->alloc(lam.size() * sizeof(double)));
    hip_check(hipMemcpy(c->d_tw, tw.data(), tw.size() * sizeof(cd), hipMemcpyHostToDevice), "upload twiddles");
    hip_check(hipMemcpy(c->d_post, post.data(), post.size() * sizeof(cd), hipMemcpyHostToDevice), "upload twiddles");
    hip_check(hipMemcpy(c->d_lam, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice), "upload eigenvalues");
    c->px.tw = c->d_tw;
    c->py.tw = c->d_tw;
    c->pz.tw = c->d_tw;
    c->py_rev.tw = c->d_tw;
    c->pz_rev.tw = c->d_tw;
    for (int a = 0; a < 3; ++a) c->st.lam[a] = c->d_lam + off[a];
    c->st.inv_ncell = 1.0 / double(g.ncell);
    if (c->dtype == INS_FP32_ALL) {
        // the all-float32 comparison mode: the same tables rounded to float32, a float32 spectrum
        std::vector<ins::cf> twf(std::max<size_t>(tw.size(), 1)), postf(post.size());
        std::vector<float> lamf(lam.size());
        for (size_t i = 0; i < tw.size(); ++i) twf[i] = ins::cf{float(tw[i].x), float(tw[i].y)};
        for (size_t i = 0; i < post.size(); ++i) postf[i] = ins::cf{float(post[i].x), float(post[i].y)};
        for (size_t i = 0; i < lam.size(); ++i) lamf[i] = float(lam[i]);
        c->d_twf = static_cast<ins::cf*>(c->alloc(twf.size() * sizeof(ins::cf)));
        c->d_postf = static_cast<ins::cf*>(c->alloc(postf.size() * sizeof(ins::cf)));
        c->d_lamf = static_cast<float*>(c->alloc(lamf.size() * sizeof(float)));
        hip_check(hipMemcpy(c->d_twf, twf.data(), twf.size() * sizeof(ins::cf), hipMemcpyHostToDevice), "upload twiddles");
        hip_check(hipMemcpy(c->d_postf, postf.data(), postf.size() * sizeof(ins::cf), hipMemcpyHostToDevice),
                  "upload twiddles");
        hip_check(hipMemcpy(c->d_lamf, lamf.data(), lamf.size() * sizeof(float), hipMemcpyHostToDevice),
                  "upload eigenvalues");
        for (ins::FftPlan* pl : {&c->px, &c->py, &c->pz, &c->py_rev, &c->pz_rev}) pl->twf = c->d_twf;
        for (int a = 0; a < 3; ++a) c->st.lamf[a] = c->d_lamf + off[a];
        c->st.inv_ncellf = float(1.0 / double(g.ncell));
        c->spec = static_cast<cd*>(c->alloc(size_t(g.batch) * g.nz * g.ny * g.sx * sizeof(ins::cf)));
        return true;
    }
    c->spec = static_cast<cd*>(c->alloc(size_t(g.batch) * g.nz * g.ny * g.sx * sizeof(cd)));
    return true;
}

ins_status ins_create(const ins_grid* grid, ins_bc bc, double nu, ins_dtype dtype, ins_ctx* out) {
    if (out) *out = nullptr;
    ins_ctx_s* c = nullptr;
    const ins_status st = guarded([&] {
        need(grid, "grid");
        need(out, "out");
        if (bc != INS_BC_PERIODIC && bc != INS_BC_WALLS_Y) raise(INS_ERR_UNSUPPORTED, "unknown boundary condition");
        const bool walls = bc == INS_BC_WALLS_Y;
        if (dtype != INS_FP64 && dtype != INS_FP32 && dtype != INS_FP32_ALL) raise(INS_ERR_INVALID, "unknown dtype");
        if (dtype == INS_FP32_ALL && walls)
            raise(INS_ERR_UNSUPPORTED, "the all-float32 comparison mode runs on the periodic grid only");
        if (grid->dim != 2 && grid->dim != 3) raise(INS_ERR_UNSUPPORTED, "dim must be 2 or 3");
        if (!(nu >= 0.0) || !std::isfinite(nu)) raise(INS_ERR_INVALID, "nu must be finite and >= 0");
        if (grid->batch < 1 || grid->batch > (1 << 20)) raise(INS_ERR_INVALID, "batch must be >= 1");
        const int d = grid->dim;
        int64_t n[3] = {grid->n[0], grid->n[1], d == 3 ? grid->n[2] : 1};
        for (int a = 0; a < d; ++a) {
            if (n[a] < 2 || n[a] > kMaxLen) raise(INS_ERR_UNSUPPORTED, "cell counts must lie in [2, 4096]");
            if (!(grid->hi[a] > grid->lo[a]) || !std::isfinite(grid->hi[a] - grid->lo[a]))
                raise(INS_ERR_INVALID, "box must have hi > lo");
        }
        if (!walls && (n[0] % 2 != 0 || n[0] < 4))
            raise(INS_ERR_UNSUPPORTED, "n_x must be even and >= 4 (real-to-complex FFT)");
        const int64_t ncell = n[0] * n[1] * n[2];
        if (ncell * d >= (int64_t(1) << 31)) raise(INS_ERR_UNSUPPORTED, "grid too large for 32-bit in-field indexing");

        std::vector<int> rx, ry, rz;
        if (!walls && (!factor(int(n[0] / 2), rx) || !factor(int(n[1]), ry) || (d == 3 && !factor(int(n[2]), rz))))
            raise(INS_ERR_UNSUPPORTED, "n_x/2, n_y, n_z must be products of 2, 3, 5, 7");

        c = new ins_ctx_s();
        c->walls = walls;
        hip_check(hipGetDevice(&c->device), "hipGetDevice");
        c->scratch = scratch_on(c->device);
        c->dtype = dtype;
        ins::Grid& g = c->g;
        g.dim = d;
        g.nx = int(n[0]);
        g.ny = int(n[1]);
        g.nz = int(n[2]);
        g.batch = int(grid->batch);
        g.ncell = ncell;
        for (int a = 0; a < 3; ++a) {
            const double h = a < d ? (grid->hi[a] - grid->lo[a]) / double(n[a]) : 1.0;
            g.ih[a] = a < d ? 1.0 / h : 0.0;
            g.ih2[a] = a < d ? 1.0 / (h * h) : 0.0;
        }
        g.nu = nu;
        g.sx = ((g.nx / 2 + 1) + 7) / 8 * 8;

        if (walls) {
            // channel grid: CG workspace instead of FFT plans and spectrum
            const size_t sb = c->scal_bytes();
            c->cg_r = static_cast<double*>(c->alloc(sb));
            c->cg_p[0] = static_cast<double*>(c->alloc(sb));
            c->cg_p[1] = static_cast<double*>(c->alloc(sb));
            c->cg_part = static_cast<double*>(c->alloc(5 * size_t(ins::cg_blocks(g)) * g.batch * sizeof(double)));
            c->cg_st = static_cast<ins::CgScal*>(c->alloc(size_t(g.batch) * sizeof(ins::CgScal)));
            c->d_ym = static_cast<double*>(c->alloc(5 * size_t(g.ny + 2) * sizeof(double)));
            upload_y_metrics(c, nullptr);
            hip_check(hipMemset(c->cg_st, 0, size_t(g.batch) * sizeof(ins::CgScal)), "hipMemset");
            hip_check(hipHostMalloc(reinterpret_cast<void**>(&c->cg_host), size_t(g.batch) * sizeof(ins::CgScal)),
                      "hipHostMalloc");
            c->p = static_cast<double*>(c->alloc(c->scal_bytes()));
            c->ry = c->alloc(c->vel_bytes());
            c->wa = c->alloc(c->vel_bytes());
            c->wb = c->alloc(c->vel_bytes());
            c->nstat = ins::stats_blocks(g);
            c->partials = static_cast<double*>(c->alloc(size_t(c->nstat) * 4 * sizeof(double)));
            // direct solver: n_x even with n_x / 2 and n_z products of 2, 3, 5, 7
            if (g.nx % 2 == 0 && g.nx >= 4 && factor(g.nx / 2, rx) && (d == 2 || factor(g.nz, rz)) &&
                g.ny <= ins::kChannelDirectMaxNy)
                c->direct_ok = setup_fft(c, rx, ry, rz, true);
            c->use_direct = c->direct_ok;
            hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
            *out = c;
            return;
        }

        setup_fft(c, rx, ry, rz, false);
        c->p = static_cast<double*>(c->alloc(c->scal_bytes()));
        c->ry = c->alloc(c->vel_bytes());
        c->wa = c->alloc(c->vel_bytes());
        c->wb = c->alloc(c->vel_bytes());
        c->nstat = ins::stats_blocks(g);
        c->partials = static_cast<double*>(c->alloc(size_t(c->nstat) * 4 * sizeof(double)));
        *out = c;
    });
    if (st != INS_OK) delete c;
    return st;
}

ins_status ins_destroy(ins_ctx ctx) {
    return guarded([&] {
        if (!ctx) return;
        (void)hipStreamSynchronize(ctx->stream);
        delete ctx;
    });
}

ins_status ins_set_stream(ins_ctx ctx, void* stream) {
    return guarded([&] {
        checked(ctx);
        ctx->collect();
        ctx->stream = static_cast<hipStream_t>(stream);
    });
}

ins_status ins_workspace_bytes(ins_ctx ctx, size_t* bytes) {
    return guarded([&] {
        checked(ctx);
        need(bytes, "bytes");
        *bytes = ctx->bytes;
    });
}

ins_status ins_rhs(ins_ctx ctx, const void* u, void* f) {
    return guarded([&] {
        checked(ctx);
        need(u, "u");
        need(f, "f");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            if (ctx->gen) {
                ctx->launch("gen_rhs", [&] {
                    return ins::launch_gen_rhs<T>(ctx->g, static_cast<const T*>(u), static_cast<T*>(f), ctx->stream);
                });
                return;
            }
            if (ctx->walls) {
                ctx->launch("wall_rhs", [&] {
                    return ins::launch_wall_rhs<T>(ctx->g, static_cast<const T*>(u), static_cast<T*>(f), ctx->stream);
                });
                return;
            }
            const T* mc = closure_at_stage<T>(ctx, static_cast<const T*>(u), nullptr);
            ctx->launch("rhs", [&] {
                return ins::launch_rhs<T>(ctx->g, static_cast<const T*>(u), static_cast<T*>(f), ctx->stream, mc);
            });
        });
    });
}

ins_status ins_divergence(ins_ctx ctx, const void* u, void* rv) {
    return guarded([&] {
        checked(ctx);
        need(u, "u");
        need(rv, "r");
        if (ctx->f32all()) {
            ctx->launch("divergence", [&] {
                return ins::launch_divergence_f32(ctx->g, static_cast<const float*>(u), static_cast<float*>(rv), ctx->stream);
            });
            return;
        }
        double* r = static_cast<double*>(rv);
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            if (ctx->gen)
                ctx->launch("gen_divergence", [&] {
                    return ins::launch_gen_divergence<T>(ctx->g, static_cast<const T*>(u), r, ctx->stream);
                });
            else if (ctx->walls)
                ctx->launch("wall_divergence", [&] {
                    return ins::launch_wall_divergence<T>(ctx->g, static_cast<const T*>(u), r, ctx->stream);
                });
            else
                ctx->launch("divergence", [&] { return ins::launch_divergence<T>(ctx->g, static_cast<const T*>(u), r, ctx->stream); });
        });
    });
}

ins_status ins_gradient(ins_ctx ctx, const void* pv, void* gout) {
    return guarded([&] {
        checked(ctx);
        need(pv, "p");
        need(gout, "g");
        if (ctx->f32all()) {
            ctx->launch("gradient", [&] {
                return ins::launch_gradient_f32(ctx->g, static_cast<const float*>(pv), static_cast<float*>(gout), ctx->stream);
            });
            return;
        }
        const double* p = static_cast<const double*>(pv);
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            if (ctx->gen)
                ctx->launch("gen_gradient", [&] { return ins::launch_gen_gradient<T>(ctx->g, p, static_cast<T*>(gout), ctx->stream); });
            else if (ctx->walls)
                ctx->launch("wall_gradient", [&] { return ins::launch_wall_gradient<T>(ctx->g, p, static_cast<T*>(gout), ctx->stream); });
            else
                ctx->launch("gradient", [&] { return ins::launch_gradient<T>(ctx->g, p, static_cast<T*>(gout), ctx->stream); });
        });
    });
}

// Pressure-point arguments are void*: float64 values, float32 in the
// all-float32 comparison mode (poisson() reinterprets them there).
ins_status ins_poisson_solve(ins_ctx ctx, const void* r, void* p) {
    return guarded([&] {
        checked(ctx);
        need(r, "r");
        need(p, "p");
        poisson(ctx, nullptr, static_cast<const double*>(r), static_cast<double*>(p));
    });
}

ins_status ins_project(ins_ctx ctx, const void* u, void* u_out, void* p_out) {
    return guarded([&] {
        checked(ctx);
        need(u, "u");
        need(u_out, "u_out");
        double* pp = p_out ? static_cast<double*>(p_out) : ctx->p;
        poisson(ctx, u, nullptr, pp);
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            apply_projection<T>(ctx, static_cast<const T*>(u), pp, static_cast<T*>(u_out));
        });
    });
}

ins_status ins_step_rk4(ins_ctx ctx, const void* u0, void* u1, double dt) {
    return guarded([&] {
        checked(ctx);
        need(u0, "u0");
        need(u1, "u1");
        check_dt(dt);
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            step_rk4<T>(ctx, static_cast<const T*>(u0), static_cast<T*>(u1), dt);
        });
    });
}

ins_status ins_rhs_vjp(ins_ctx ctx, const void* u, const void* fbar, void* ubar) {
    return guarded([&] {
        checked(ctx);
        need(u, "u");
        need(fbar, "fbar");
        need(ubar, "ubar");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            if (ctx->gen) {
                ctx->launch("gen_rhs_vjp", [&] {
                    return ins::launch_gen_rhs_vjp<T>(ctx->g, static_cast<const T*>(u), static_cast<const T*>(fbar),
                                                      static_cast<T*>(ubar), ctx->stream);
                });
                return;
            }
            if (ctx->walls) {
                ctx->launch("wall_rhs_vjp", [&] {
                    return ins::launch_wall_rhs_vjp<T>(ctx->g, static_cast<const T*>(u), static_cast<const T*>(fbar),
                                                       static_cast<T*>(ubar), ctx->stream);
                });
                return;
            }
            ctx->launch("rhs_vjp", [&] {
                return ins::launch_rhs_vjp<T>(ctx->g, static_cast<const T*>(u), static_cast<const T*>(fbar),
                                              static_cast<T*>(ubar), ctx->stream);
            });
            if (ctx->clos_on) {
                closure_forward<T>(ctx, static_cast<const T*>(u), static_cast<T*>(ctx->mclos));
                closure_backward<T>(ctx, static_cast<const T*>(fbar), static_cast<T*>(ubar));
            }
        });
    });
}

ins_status ins_divergence_vjp(ins_ctx ctx, const double* rbar, void* ubar) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_divergence_vjp");
        need(rbar, "rbar");
        need(ubar, "ubar");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            if (ctx->gen)
                ctx->launch("gen_divergence_vjp", [&] { return ins::launch_gen_div_vjp<T>(ctx->g, rbar, static_cast<T*>(ubar), ctx->stream); });
            else if (ctx->walls)
                ctx->launch("wall_divergence_vjp", [&] { return ins::launch_wall_div_vjp<T>(ctx->g, rbar, static_cast<T*>(ubar), ctx->stream); });
            else
                ctx->launch("divergence_vjp", [&] { return ins::launch_div_vjp<T>(ctx->g, rbar, static_cast<T*>(ubar), ctx->stream); });
        });
    });
}

ins_status ins_gradient_vjp(ins_ctx ctx, const void* gbar, double* pbar) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_gradient_vjp");
        need(gbar, "gbar");
        need(pbar, "pbar");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            if (ctx->gen)
                ctx->launch("gen_gradient_vjp", [&] { return ins::launch_gen_grad_vjp<T>(ctx->g, static_cast<const T*>(gbar), pbar, ctx->stream); });
            else if (ctx->walls)
                ctx->launch("wall_gradient_vjp", [&] { return ins::launch_wall_grad_vjp<T>(ctx->g, static_cast<const T*>(gbar), pbar, ctx->stream); });
            else
                ctx->launch("gradient_vjp", [&] { return ins::launch_grad_vjp<T>(ctx->g, static_cast<const T*>(gbar), pbar, ctx->stream); });
        });
    });
}

ins_status ins_poisson_solve_vjp(ins_ctx ctx, const void* pbarv, void* rbarv) {
    if (!ctx || !(ctx->walls || ctx->gen)) return ins_poisson_solve(ctx, pbarv, rbarv);
    const double* pbar = static_cast<const double*>(pbarv);
    double* rbar = static_cast<double*>(rbarv);
    return guarded([&] {
        checked(ctx);
        need(pbar, "pbar");
        need(rbar, "rbar");
        // channel: the solve is p = S^+ Omega_p (r - mean_w(r)) with S = -Omega_p D G
        // symmetric (zero-mean p), so its transpose is
        // rbar = Omega_p (t - mean_w(t)), t = S^+ (mean(pbar) - pbar)
        if (ctx->use_direct) {
            direct_solve(ctx, nullptr, pbar, rbar, 3);
            return;
        }
        cg_solve(ctx, nullptr, pbar, rbar, 3);
        ctx->launch("cg_weighted_center", [&] {
            return ins::launch_cg_weighted_center(ctx->g, rbar, ctx->cg_part, ctx->wsum, ctx->stream);
        });
    });
}

ins_status ins_project_vjp(ins_ctx ctx, const void* ubar_out, void* ubar) {
    if (!ctx || !(ctx->walls || ctx->gen)) return ins_project(ctx, ubar_out, ubar, nullptr);
    return guarded([&] {
        checked(ctx);
        need(ubar_out, "ubar_out");
        need(ubar, "ubar");
        // channel: P^T = Omega_u P Omega_u^{-1}
        poisson(ctx, ubar_out, nullptr, ctx->p, true);
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            apply_projection<T>(ctx, static_cast<const T*>(ubar_out), ctx->p, static_cast<T*>(ubar), true);
        });
    });
}

ins_status ins_step_rk4_vjp(ins_ctx ctx, const void* u0, const void* u1bar, void* u0bar, double dt) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_step_rk4_vjp");
        need(u0, "u0");
        need(u1bar, "u1bar");
        need(u0bar, "u0bar");
        check_dt(dt);
        if (u0bar == u0 || u0bar == u1bar) raise(INS_ERR_INVALID, "u0bar must not alias u0 or u1bar");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            step_rk4_vjp<T>(ctx, static_cast<const T*>(u0), static_cast<const T*>(u1bar), static_cast<T*>(u0bar), dt);
        });
    });
}

ins_status ins_step_wray3(ins_ctx ctx, const void* u0, void* u1, double dt) {
    return guarded([&] {
        checked(ctx);
        need(u0, "u0");
        need(u1, "u1");
        check_dt(dt);
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            step_wray3<T>(ctx, static_cast<const T*>(u0), static_cast<T*>(u1), dt);
        });
    });
}

ins_status ins_step_wray3_vjp(ins_ctx ctx, const void* u0, const void* u1bar, void* u0bar, double dt) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_step_wray3_vjp");
        need(u0, "u0");
        need(u1bar, "u1bar");
        need(u0bar, "u0bar");
        check_dt(dt);
        if (u0bar == u0 || u0bar == u1bar) raise(INS_ERR_INVALID, "u0bar must not alias u0 or u1bar");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            step_wray3_vjp<T>(ctx, static_cast<const T*>(u0), static_cast<const T*>(u1bar), static_cast<T*>(u0bar),
                              dt);
        });
    });
}

int ins_scheme_stage_count(int scheme) { return scheme == INS_RK4 ? 3 : (scheme == INS_WRAY3 ? 2 : -1); }

ins_status ins_step_save(ins_ctx ctx, int scheme, const void* u0, void* u1, double dt, void* stages,
                         double* pstages) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_step_save");
        need(u0, "u0");
        need(u1, "u1");
        need(stages, "stages");
        need(pstages, "pstages");
        check_dt(dt);
        const int ns = ins_scheme_stage_count(scheme);
        if (ns < 0) raise(INS_ERR_INVALID, "unknown scheme");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            const size_t nv = ctx->vel_bytes() / sizeof(T), np = ctx->scal_bytes() / sizeof(double);
            Stages<T> S{};
            for (int i = 0; i < ns; ++i) {
                S.w[i] = static_cast<T*>(stages) + i * nv;
                S.p[i] = pstages + i * np;
            }
            if (scheme == INS_RK4)
                step_rk4<T>(ctx, static_cast<const T*>(u0), static_cast<T*>(u1), dt, &S);
            else
                step_wray3<T>(ctx, static_cast<const T*>(u0), static_cast<T*>(u1), dt, &S);
        });
    });
}

ins_status ins_step_vjp_saved(ins_ctx ctx, int scheme, const void* u0, const void* stages, const double* pstages,
                              const void* u1bar, void* u0bar, double dt) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_step_vjp_saved");
        need(u0, "u0");
        need(stages, "stages");
        need(pstages, "pstages");
        need(u1bar, "u1bar");
        need(u0bar, "u0bar");
        check_dt(dt);
        const int ns = ins_scheme_stage_count(scheme);
        if (ns < 0) raise(INS_ERR_INVALID, "unknown scheme");
        if (u0bar == u0 || u0bar == u1bar || u0bar == stages) raise(INS_ERR_INVALID, "u0bar must not alias an input");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            const size_t nv = ctx->vel_bytes() / sizeof(T), np = ctx->scal_bytes() / sizeof(double);
            Stages<T> S{};
            for (int i = 0; i < ns; ++i) {
                S.w[i] = const_cast<T*>(static_cast<const T*>(stages)) + i * nv;
                S.p[i] = const_cast<double*>(pstages) + i * np;
            }
            if (scheme == INS_RK4)
                step_rk4_reverse<T>(ctx, static_cast<const T*>(u0), S, static_cast<const T*>(u1bar),
                                    static_cast<T*>(u0bar), dt);
            else
                step_wray3_reverse<T>(ctx, static_cast<const T*>(u0), S, static_cast<const T*>(u1bar),
                                      static_cast<T*>(u0bar), dt);
        });
    });
}

ins_status ins_cg_set(ins_ctx ctx, double rtol, int maxiter, int check_every) {
    return guarded([&] {
        checked(ctx);
        if (!ctx->walls && !ctx->gen) raise(INS_ERR_UNSUPPORTED, "the uniform periodic grid solves by FFT, not CG");
        if (!(rtol >= 0.0) || !std::isfinite(rtol)) raise(INS_ERR_INVALID, "rtol must be finite and >= 0");
        if (maxiter < 1 || check_every < 0) raise(INS_ERR_INVALID, "maxiter must be >= 1 and check_every >= 0");
        ctx->cg_rtol = rtol;
        ctx->cg_maxiter = maxiter;
        ctx->cg_check = check_every;
    });
}

// Checks and stores the n_a + 1 faces of direction a (host copy).
void store_faces(ins_ctx c, int a, const double* faces) {
    const int n = a == 0 ? c->g.nx : (a == 1 ? c->g.ny : c->g.nz);
    for (int j = 0; j <= n; ++j)
        if (!std::isfinite(faces[j])) raise(INS_ERR_INVALID, "face coordinates must be finite");
    for (int j = 0; j < n; ++j)
        if (!(faces[j + 1] > faces[j])) raise(INS_ERR_INVALID, "face coordinates must increase strictly");
    c->faces[a].assign(faces, faces + n + 1);
}

ins_status ins_set_y_faces(ins_ctx ctx, const double* faces) {
    return guarded([&] {
        checked(ctx);
        need(faces, "faces");
        if (!ctx->walls) raise(INS_ERR_UNSUPPORTED, "a stretched y grid needs the channel (INS_BC_WALLS_Y)");
        store_faces(ctx, 1, faces);
        upload_y_metrics(ctx, faces);
        if (ctx->gen) upload_gen_metrics(ctx);
    });
}

ins_status ins_set_faces(ins_ctx ctx, int axis, const double* faces) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_set_faces");
        need(faces, "faces");
        if (axis < 0 || axis >= ctx->g.dim) raise(INS_ERR_INVALID, "axis must be 0 .. dim - 1");
        if (ctx->walls && axis == 1) {
            store_faces(ctx, 1, faces);
            upload_y_metrics(ctx, faces);
            if (ctx->gen) upload_gen_metrics(ctx);
            return;
        }
        if (ctx->clos_on) raise(INS_ERR_UNSUPPORTED, "closures need the uniform periodic grid: clear the closure first");
        store_faces(ctx, axis, faces);
        if (!ctx->gen) enter_gen(ctx);
        upload_gen_metrics(ctx);
    });
}

ins_status ins_set_body_force(ins_ctx ctx, const double* force) {
    return guarded([&] {
        checked(ctx);
        need(force, "force");
        if (!ctx->walls) raise(INS_ERR_UNSUPPORTED, "the body force is a channel (INS_BC_WALLS_Y) feature");
        for (int a = 0; a < ctx->g.dim; ++a)
            if (!std::isfinite(force[a])) raise(INS_ERR_INVALID, "force components must be finite");
        for (int a = 0; a < 3; ++a) ctx->g.force[a] = a < ctx->g.dim ? force[a] : 0.0;
    });
}

ins_status ins_cg_info(ins_ctx ctx, int* iterations, double* relres) {
    return guarded([&] {
        checked(ctx);
        need(iterations, "iterations");
        need(relres, "relres");
        if (!ctx->walls && !ctx->gen) raise(INS_ERR_UNSUPPORTED, "the uniform periodic grid solves by FFT, not CG");
        cg_all_done(ctx);
        int it = 0;
        double rr = 0.0;
        for (int b = 0; b < ctx->g.batch; ++b) {
            it = std::max(it, ctx->cg_host[b].it);
            rr = std::max(rr, ctx->cg_host[b].relres);
        }
        *iterations = it;
        *relres = rr;
    });
}

ins_status ins_set_pressure_solver(ins_ctx ctx, int solver) {
    return guarded([&] {
        checked(ctx);
        if (solver != INS_PRESSURE_AUTO && solver != INS_PRESSURE_FFT && solver != INS_PRESSURE_CG)
            raise(INS_ERR_INVALID, "unknown pressure solver");
        if (ctx->gen) {
            if (solver == INS_PRESSURE_FFT) raise(INS_ERR_UNSUPPORTED, "a stretched grid solves by CG, not FFT");
            return;
        }
        if (!ctx->walls) {
            if (solver == INS_PRESSURE_CG) raise(INS_ERR_UNSUPPORTED, "the periodic grid solves by FFT, not CG");
            return;
        }
        if (solver == INS_PRESSURE_FFT && !ctx->direct_ok)
            raise(INS_ERR_UNSUPPORTED,
                  "the channel's FFT solve needs n_x even, n_x/2 and n_z products of 2, 3, 5, 7 and n_y <= 2048");
        ctx->use_direct = solver == INS_PRESSURE_CG ? false : ctx->direct_ok;
    });
}

ins_status ins_get_pressure_solver(ins_ctx ctx, int* solver) {
    return guarded([&] {
        checked(ctx);
        need(solver, "solver");
        *solver = (ctx->gen || (ctx->walls && !ctx->use_direct)) ? INS_PRESSURE_CG : INS_PRESSURE_FFT;
    });
}

ins_status ins_face_filter(ins_ctx ctx, const void* u, int factor, void* u_coarse) {
    return guarded([&] {
        checked(ctx);
        periodic_only(ctx, "ins_face_filter");
        need(u, "u");
        need(u_coarse, "u_coarse");
        const ins::Grid& g = ctx->g;
        if (factor < 1 || g.nx % factor || g.ny % factor || (g.dim == 3 && g.nz % factor))
            raise(INS_ERR_INVALID, "every cell count must be divisible by the filter factor");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            ctx->launch("face_filter", [&] {
                return ins::launch_face_filter<T>(g, factor, static_cast<const T*>(u), static_cast<T*>(u_coarse), ctx->stream);
            });
        });
    });
}

ins_status ins_energy_spectrum(ins_ctx ctx, const void* u, double* e, int nbins) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_energy_spectrum");
        periodic_only(ctx, "ins_energy_spectrum");
        need(u, "u");
        need(e, "e");
        if (nbins < 1) raise(INS_ERR_INVALID, "nbins must be >= 1");
        const ins::Grid& g = ctx->g;
        ctx->launch("fill_zero", [&] { return ins::launch_fill_zero(e, size_t(nbins) * g.batch, ctx->stream); });
        for (int a = 0; a < g.dim; ++a) {
            with_type(ctx, [&](auto tag) {
                using T = decltype(tag);
                ctx->launch("fft_x_fwd", [&] {
                    return ins::launch_fft_x_fwd<T>(g, static_cast<const T*>(u), nullptr, ctx->spec, ctx->px, ctx->d_post,
                                                    ctx->lnl_x, ctx->stream, a);
                });
            });
            ctx->launch("fft_y_fwd", [&] { return ins::launch_fft_strided(g, ctx->spec, ctx->py, ctx->py, 1, 0, ctx->lnl_y, ctx->st, ctx->stream); });
            if (g.dim == 3)
                ctx->launch("fft_z_fwd", [&] { return ins::launch_fft_strided(g, ctx->spec, ctx->pz, ctx->pz, 2, 0, ctx->lnl_z, ctx->st, ctx->stream); });
            ctx->launch("spectrum_bins", [&] { return ins::launch_spectrum_bins(g, ctx->spec, e, nbins, ctx->stream); });
        }
    });
}

ins_status ins_closure_set(ins_ctx ctx, const float* params) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_closure_set");
        periodic_only(ctx, "ins_closure_set");
        if (!params) {
            if (ctx->clos_kind == 1) {
                ctx->clos_on = false;
                ctx->clos_kind = 0;
            }
            return;
        }
        const ins::Grid& g = ctx->g;
        if (g.dim != 3) raise(INS_ERR_UNSUPPORTED, "the closure is a 3D convolutional network");
        if (g.nx % 32 != 0) raise(INS_ERR_UNSUPPORTED, "the closure needs n_x divisible by 32");
        closure_alloc(ctx);
        hip_check(hipMemcpyAsync(ctx->theta, params, kClosParams * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream),
                  "copy closure parameters");
        const int cin[3] = {3, 32, 32}, cout[3] = {32, 32, 3}, cinp[3] = {8, 32, 32}, ntf[3] = {2, 2, 1},
                  coutp[3] = {32, 32, 8}, ntd[3] = {1, 2, 2};
        const int woff[3] = {kW1, kW2, kW3};
        for (int l = 0; l < 3; ++l) {
            ctx->launch("cnn_pack_weights", [&] {
                return ins::launch_closure_pack_weights(ctx->theta + woff[l], cin[l], cout[l], cinp[l], ntf[l], ctx->wf[l],
                                                        coutp[l], ntd[l], ctx->wd[l], ctx->stream);
            });
        }
        ctx->clos_on = true;
        ctx->clos_kind = 1;
    });
}

ins_status ins_eddy_set(ins_ctx ctx, double cs, double delta) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_eddy_set");
        periodic_only(ctx, "ins_eddy_set");
        if (!(cs >= 0.0) || !std::isfinite(cs)) raise(INS_ERR_INVALID, "cs must be finite and >= 0");
        if (!std::isfinite(delta)) raise(INS_ERR_INVALID, "delta must be finite");
        if (cs == 0.0) {
            if (ctx->clos_kind == 2) {
                ctx->clos_on = false;
                ctx->clos_kind = 0;
            }
            return;
        }
        const ins::Grid& g = ctx->g;
        double width = delta;
        if (!(width > 0.0)) {  // geometric mean of the spacings
            double prod = 1.0;
            for (int a = 0; a < g.dim; ++a) prod /= g.ih[a];
            width = std::pow(prod, 1.0 / g.dim);
        }
        eddy_alloc(ctx);
        ctx->eddy_c2 = (cs * width) * (cs * width);
        ctx->clos_on = true;
        ctx->clos_kind = 2;
    });
}

ins_status ins_eddy_forward(ins_ctx ctx, const void* u, void* m) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_eddy_forward");
        periodic_only(ctx, "ins_eddy_forward");
        need(u, "u");
        need(m, "m");
        if (ctx->clos_kind != 2) raise(INS_ERR_INVALID, "no eddy-viscosity closure has been set");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            closure_forward<T>(ctx, static_cast<const T*>(u), static_cast<T*>(m));
        });
    });
}

ins_status ins_eddy_backward(ins_ctx ctx, const void* u, const void* mbar, void* ubar) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_eddy_backward");
        periodic_only(ctx, "ins_eddy_backward");
        need(u, "u");
        need(mbar, "mbar");
        need(ubar, "ubar");
        if (ctx->clos_kind != 2) raise(INS_ERR_INVALID, "no eddy-viscosity closure has been set");
        if (ubar == u || ubar == mbar) raise(INS_ERR_INVALID, "ubar must not alias u or mbar");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            const size_t nv = ctx->vel_bytes() / sizeof(T);
            ctx->launch("fill_zero", [&] {
                return sizeof(T) == 8 ? ins::launch_fill_zero(reinterpret_cast<double*>(ubar), nv, ctx->stream)
                                      : ins::launch_fill_zero_f(reinterpret_cast<float*>(ubar), nv, ctx->stream);
            });
            closure_forward<T>(ctx, static_cast<const T*>(u), static_cast<T*>(ctx->mclos));
            closure_backward<T>(ctx, static_cast<const T*>(mbar), static_cast<T*>(ubar));
        });
    });
}

ins_status ins_closure_grad(ins_ctx ctx, float* params_bar) {
    return guarded([&] {
        checked(ctx);
        need(params_bar, "params_bar");
        if (!ctx->clos_alloc) raise(INS_ERR_INVALID, "no closure has been set");
        hip_check(hipMemcpyAsync(params_bar, ctx->theta_bar, kClosParams * sizeof(float), hipMemcpyDeviceToDevice,
                                 ctx->stream),
                  "copy closure gradient");
        ctx->launch("fill_zero", [&] { return ins::launch_fill_zero_f(ctx->theta_bar, kClosParams, ctx->stream); });
    });
}

ins_status ins_cnn_forward(ins_ctx ctx, const void* u, void* m) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_cnn_forward");
        periodic_only(ctx, "ins_cnn_forward");
        need(u, "u");
        need(m, "m");
        if (ctx->clos_kind != 1) raise(INS_ERR_INVALID, "no learned closure has been set");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            closure_forward<T>(ctx, static_cast<const T*>(u), static_cast<T*>(m), false);
        });
    });
}

ins_status ins_cnn_backward(ins_ctx ctx, const void* u, const void* mbar, void* ubar, float* params_bar) {
    return guarded([&] {
        checked(ctx);
        no_f32all(ctx, "ins_cnn_backward");
        periodic_only(ctx, "ins_cnn_backward");
        need(u, "u");
        need(mbar, "mbar");
        need(ubar, "ubar");
        need(params_bar, "params_bar");
        if (ctx->clos_kind != 1) raise(INS_ERR_INVALID, "no learned closure has been set");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            const size_t nv = ctx->vel_bytes() / sizeof(T);
            ctx->launch("fill_zero", [&] {
                return sizeof(T) == 8 ? ins::launch_fill_zero(reinterpret_cast<double*>(ubar), nv, ctx->stream)
                                      : ins::launch_fill_zero_f(reinterpret_cast<float*>(ubar), nv, ctx->stream);
            });
            ctx->launch("fill_zero", [&] { return ins::launch_fill_zero_f(ctx->theta_bar, kClosParams, ctx->stream); });
            closure_forward<T>(ctx, static_cast<const T*>(u), static_cast<T*>(ctx->mclos));
            closure_backward<T>(ctx, static_cast<const T*>(mbar), static_cast<T*>(ubar));
        });
        hip_check(hipMemcpyAsync(params_bar, ctx->theta_bar, kClosParams * sizeof(float), hipMemcpyDeviceToDevice,
                                 ctx->stream),
                  "copy closure gradient");
        ctx->launch("fill_zero", [&] { return ins::launch_fill_zero_f(ctx->theta_bar, kClosParams, ctx->stream); });
    });
}

ins_status ins_cnn_saved(ins_ctx ctx, int which, void* out) {
    return guarded([&] {
        checked(ctx);
        need(out, "out");
        if (ctx->clos_kind != 1 || !ctx->clos_alloc) raise(INS_ERR_INVALID, "no learned closure has been set");
        const size_t n = size_t(ctx->g.ncell) * ctx->g.batch;
        const void* src = nullptr;
        size_t bytes = 0;
        switch (which) {
            case 0: src = ctx->x0, bytes = n * 8 * 2; break;
            case 1: src = ctx->z1, bytes = n * 32 * 4; break;
            case 2: src = ctx->a1, bytes = n * 32 * 2; break;
            case 3: src = ctx->z2, bytes = n * 32 * 4; break;
            case 4: src = ctx->a2, bytes = n * 32 * 2; break;
            case 5: src = ctx->gm, bytes = n * 8 * 2; break;
            case 6: src = ctx->gz2, bytes = n * 32 * 2; break;
            case 7: src = ctx->gz1, bytes = n * 32 * 2; break;
            case 8: src = ctx->mclos, bytes = ctx->vel_bytes(); break;
            default: raise(INS_ERR_INVALID, "ins_cnn_saved: which must be 0..8");
        }
        hip_check(hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToDevice, ctx->stream), "copy closure tensor");
    });
}

ins_status ins_stats(ins_ctx ctx, const void* u, double out[4]) {
    return guarded([&] {
        checked(ctx);
        need(u, "u");
        need(out, "out");
        with_type(ctx, [&](auto tag) {
            using T = decltype(tag);
            ctx->launch("stats", [&] {
                return ins::launch_stats<T>(ctx->g, static_cast<const T*>(u), ctx->partials, ctx->nstat, ctx->stream);
            });
        });
        std::vector<double> h(size_t(ctx->nstat) * 4);
        hip_check(hipMemcpyAsync(h.data(), ctx->partials, h.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
                  "copy partials");
        hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        double s2 = 0.0, mu = 0.0, md = 0.0, nf = 0.0;
        for (int b = 0; b < ctx->nstat; ++b) {
            s2 += h[4 * b];
            mu = std::max(mu, h[4 * b + 1]);
            md = std::max(md, h[4 * b + 2]);
            nf += h[4 * b + 3];
        }
        out[0] = 0.5 * s2 / (double(ctx->g.ncell) * ctx->g.batch);
        out[1] = mu;
        out[2] = md;
        out[3] = nf == 0.0 ? 1.0 : 0.0;
    });
}

ins_status ins_stats_noalloc(ins_ctx ctx, const void* u, double* out) {
    return guarded([&] {
        checked(ctx);
        need(u, "u");
        need(out, "out");
        if (size_t(4) * size_t(ins::stats_capped_blocks(ctx->g)) > kScratchDoubles)
            raise(INS_ERR_UNSUPPORTED, "ins_stats_noalloc: partials exceed the fixed scratch");
        // launched directly (no profiling events): this call creates nothing
        hipError_t e;
        if (ctx->dtype == INS_FP64)
            e = ins::launch_stats_capped<double>(ctx->g, static_cast<const double*>(u), ctx->scratch, out, ctx->stream);
        else
            e = ins::launch_stats_capped<float>(ctx->g, static_cast<const float*>(u), ctx->scratch, out, ctx->stream);
        if (e != hipSuccess) raise(INS_ERR_HIP, std::string("stats_capped: ") + hipGetErrorString(e));
    });
}

ins_status ins_stream_copy(ins_ctx ctx, const void* src, void* dst, size_t nbytes) {
    return guarded([&] {
        checked(ctx);
        need(src, "src");
        need(dst, "dst");
        if (nbytes % 16 != 0) raise(INS_ERR_INVALID, "nbytes must be a multiple of 16");
        ctx->launch("stream_copy", [&] { return ins::launch_stream_copy(src, dst, nbytes, ctx->stream); });
    });
}

ins_status ins_profile_enable(ins_ctx ctx, int enable) {
    return guarded([&] {
        checked(ctx);
        ctx->prof = enable != 0;
    });
}

ins_status ins_profile_reset(ins_ctx ctx) {
    return guarded([&] {
        checked(ctx);
        ctx->collect();
        ctx->totals.clear();
        ctx->order.clear();
    });
}

ins_status ins_profile_count(ins_ctx ctx, int* count) {
    return guarded([&] {
        checked(ctx);
        need(count, "count");
        ctx->collect();
        *count = int(ctx->order.size());
    });
}

ins_status ins_profile_read(ins_ctx ctx, int i, char* name, size_t name_len, int64_t* launches, double* total_ms) {
    return guarded([&] {
        checked(ctx);
        ctx->collect();
        if (i < 0 || i >= int(ctx->order.size())) raise(INS_ERR_INVALID, "profile index out of range");
        const std::string& nm = ctx->order[size_t(i)];
        if (name && name_len > 0) {
            std::strncpy(name, nm.c_str(), name_len - 1);
            name[name_len - 1] = '\0';
        }
        const auto& tot = ctx->totals[nm];
        if (launches) *launches = tot.first;
        if (total_ms) *total_ms = tot.second;
    });
}

}  // extern "C"
