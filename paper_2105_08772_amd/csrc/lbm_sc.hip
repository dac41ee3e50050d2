// Host side of the C ABI declared in include/lbm_sc.h: configuration checks, the flat-interface
// coexistence rule, device memory, the step loop and the observables assembly.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm_sc.h"
#include "kernels.hpp"

namespace {

// Message of the last failure on this thread, in a fixed buffer so that recording an error
// allocates nothing.
thread_local char g_err[512] = "no error";

const char* const SHAPE_MSG =
    "unsupported launch shape (tile_x 64: waves 4 with rows 1, 2, 4, or waves 8 with rows 1, 2 and no "
    "prefetch; tile_x 32: rows 1, 2 (waves 8: no prefetch); tile_x 0: no prefetch, waves 8 with rows 2, 4 or 8, or waves 4 with rows 4)";

const char* const SHAPE2_MSG =
    "unsupported two-step launch shape (tile_x 64 with rows 1 and waves 8, tile_x 32 with rows 2 and "
    "waves 8, or without prefetch tile_x 32 with rows 2 and waves 4 or tile_x 64 with rows 2 and "
    "waves 16)";

int fail(int code, const char* msg)
{
    std::snprintf(g_err, sizeof(g_err), "%s", msg);
    return code;
}

int fail(int code, const std::string& msg) { return fail(code, msg.c_str()); }

int fail_hip(const char* what, hipError_t e)
{
    return fail(LBM_SC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return fail_hip(#expr, e_); \
    } while (0)

// ------------------------------------------------------------------------------------------
// Equation of state (Eq. bulkp with e_2 = 1, c_s^2 = 1/3)
// ------------------------------------------------------------------------------------------

constexpr double CS2 = 1.0 / 3.0;

double psi_h(double n, int kind) { return kind == 0 ? std::exp(-1.0 / n) : -std::expm1(-n); }
double dpsi_h(double n, int kind)
{
    return kind == 0 ? std::exp(-1.0 / n) / (n * n) : std::exp(-n);
}
double dlogpsi_h(double n, int kind) { return kind == 0 ? 1.0 / (n * n) : 1.0 / std::expm1(n); }
double P_h(double n, double G, int kind)
{
    const double p = psi_h(n, kind);
    return n * CS2 + 0.5 * G * CS2 * p * p;
}
double dP_h(double n, double G, int kind) { return CS2 + G * CS2 * psi_h(n, kind) * dpsi_h(n, kind); }

double gc_h(int kind) { return kind == 0 ? -std::exp(2.0) : -4.0; }
double nc_h(int kind) { return kind == 0 ? 1.0 : std::log(2.0); }

template <typename F>
bool bisect(F f, double lo, double hi, double& root)
{
    double flo = f(lo), fhi = f(hi);
    if (!(flo * fhi <= 0.0)) return false;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        const double fm = f(mid);
        if ((fm <= 0.0) == (flo <= 0.0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    root = 0.5 * (lo + hi);
    return true;
}

// Adaptive Simpson quadrature.
template <typename F>
double simpson_rec(F& f, double a, double b, double fa, double fm, double fb, double whole,
                   double tol, int depth)
{
    const double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
    const double flm = f(lm), frm = f(rm);
    const double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
    const double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
    const double d = left + right - whole;
    if (depth <= 0 || std::fabs(d) <= 15.0 * tol) return left + right + d / 15.0;
    return simpson_rec(f, a, m, fa, flm, fm, left, 0.5 * tol, depth - 1) +
           simpson_rec(f, m, b, fm, frm, fb, right, 0.5 * tol, depth - 1);
}

template <typename F>
double integrate(F f, double a, double b, double tol)
{
    // split into panels so that the recursion starts resolved
    const int panels = 64;
    double total = 0.0;
    for (int k = 0; k < panels; ++k) {
        const double x0 = a + (b - a) * k / panels, x1 = a + (b - a) * (k + 1) / panels;
        const double f0 = f(x0), f1 = f(x1), fm = f(0.5 * (x0 + x1));
        const double whole = (x1 - x0) / 6.0 * (f0 + 4.0 * fm + f1);
        total += simpson_rec(f, x0, x1, f0, fm, f1, whole, tol / panels, 40);
    }
    return total;
}

struct Coex {
    double ng, nl, p0;
};

// Leading-order flat coexistence: P(n_g) = P(n_l) = p0, int (p0 - P) psi'/psi dn = 0.
bool coexistence(int kind, double ratio, Coex& out)
{
    if (!(ratio > 1.0)) return false;
    const double G = ratio * gc_h(kind), nc = nc_h(kind);
    double sg, sl;
    auto dP = [&](double n) { return dP_h(n, G, kind); };
    if (!bisect(dP, 1e-3, nc, sg) || !bisect(dP, nc, 50.0, sl)) return false;
    auto roots = [&](double p0, double& ng, double& nl) {
        auto h = [&](double n) { return P_h(n, G, kind) - p0; };
        return bisect(h, std::fmin(1e-9, 0.5 * p0), sg, ng) && bisect(h, sl, 200.0, nl);
    };
    auto residual = [&](double p0, bool& ok) {
        double ng, nl;
        ok = roots(p0, ng, nl);
        if (!ok) return 0.0;
        auto integrand = [&](double n) { return (p0 - P_h(n, G, kind)) * dlogpsi_h(n, kind); };
        return integrate(integrand, ng, nl, 1e-15);
    };
    const double p_hi = P_h(sg, G, kind);
    const double p_lo = std::fmax(P_h(sl, G, kind), 0.0);
    const double eps = 1e-9 * (p_hi - p_lo);
    bool ok;
    double hi = p_hi - eps, r_hi = residual(hi, ok);
    if (!ok) return false;
    double lo = -1.0;
    for (int k = 1; k < 60; ++k) {
        // geometric steps away from the top of the coexistence range
        const double frac = std::pow(10.0, -9.0 + 9.0 * k / 59.0);
        double p = p_hi - (p_hi - p_lo) * frac;
        if (k == 59) p = p_lo + eps;
        const double r = residual(p, ok);
        if (!ok) return false;
        if ((r > 0.0) != (r_hi > 0.0)) {
            lo = p;
            break;
        }
        hi = p;
        r_hi = r;
    }
    if (lo < 0.0) return false;
    double p0;
    auto res = [&](double p) {
        bool okk;
        return residual(p, okk);
    };
    if (!bisect(res, lo, hi, p0)) return false;
    double ng, nl;
    if (!roots(p0, ng, nl)) return false;
    out = {ng, nl, p0};
    return true;
}

}  // namespace

struct lbm_sc {
    lbm_sc_config cfg;
    lbm::BoxDesc box;
    lbm::StepShape shape;
    lbm::InitDesc init;
    bool fp32 = false;    // populations stored as float (shifted)
    bool math64 = false;  // with fp32: step arithmetic in double precision
    size_t elem = 8;
    void* pop[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t step = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool own_pop = true;       // false: the population buffers belong to the caller
    int dev = 0;               // HIP device of the box (its observation workspace)
    double* d_uprev = nullptr; // 3N doubles: velocity of the last observation
    double* d_parts = nullptr; // OBS_BLOCKS * OBS_PARTS
    double* d_small = nullptr; // scalars (OBS_PARTS) + probes (4) + dither step counts (2 x u32)
    double* d_prof = nullptr;  // 4 * Lmax
    int has_prev = 0;
    double mass0 = 0.0;
    double G = 0.0, Gc = 0.0;
    int64_t device_bytes = 0;
    int graph_steps = 64;              // steps per captured chunk (even; 0: no graph)
    int spp = 1;                       // time steps per kernel pass (2: FP32, tau = 1 only)
    lbm::StepShape shape2;             // launch shape of the two-step kernel (spp = 2)
    hipGraphExec_t graph = nullptr;    // graph_len steps captured from buffer graph_cur
    int graph_len = 0;
    int graph_cur = 0;
    std::vector<lbm_sc_group*> groups;  // groups whose box list holds this box
};

namespace {

// Row pitch of the stored populations. Padded rows (the default): nx rounded up to whole 128-byte
// lines, so that every row starts on a line and the step kernel writes complete lines (it fills
// the padding of the last line of each row, which nothing reads); x-y tiles need this. Packed
// rows: pitch nx, for full-row tiles, whose lane window the kernel aligns with the line grid
// itself, so that no lanes idle over padding.
unsigned row_pitch(int nx, size_t elem, int packed)
{
    if (packed) return (unsigned)nx;
    const unsigned per_line = (unsigned)(128 / elem);
    return ((unsigned)nx + per_line - 1) / per_line * per_line;
}

// Population pitch: elements between the 19 population planes of one z-plane, the plane px * ny
// rounded up to 64 elements and, for planes of 64 KiB or more, padded by about a 19th of the
// plane (rounded down to 256 B), so that the 19 planes start at offsets spread evenly modulo the
// plane size instead of coinciding modulo a large power of two (measured at 256^3 against a
// 256-byte pad: FP32 step 0.489 -> 0.487 ms, FP64 0.962 -> 0.937 ms).
unsigned long long population_pitch(unsigned long long pxy, size_t elem)
{
    unsigned long long s = (pxy + 63ull) / 64ull * 64ull;
    const unsigned long long bytes = s * elem;
    if (bytes >= (64ull << 10)) s += bytes / 19ull / 256ull * 256ull / elem;
    return s;
}

int validate(const lbm_sc_config* c)
{
    if (!c) return fail(LBM_SC_EINVAL, "cfg is NULL");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(LBM_SC_EINVAL, "box sizes must be >= 1");
    const double nodes = (double)c->nx * c->ny * c->nz;
    if (nodes > 2147483648.0) return fail(LBM_SC_EINVAL, "box has more than 2^31 nodes");
    if (c->psi != LBM_SC_PSI_EXP && c->psi != LBM_SC_PSI_ONEMINUS)
        return fail(LBM_SC_EINVAL, "psi must be LBM_SC_PSI_EXP or LBM_SC_PSI_ONEMINUS");
    if (c->geom < LBM_SC_DROPLET || c->geom > LBM_SC_FROM_HOST)
        return fail(LBM_SC_EINVAL, "unknown geom");
    if (c->prec != LBM_SC_FP64 && c->prec != LBM_SC_FP32_SHIFTED && c->prec != LBM_SC_FP32_SHIFTED_MATH64)
        return fail(LBM_SC_EINVAL,
                    "prec must be LBM_SC_FP64, LBM_SC_FP32_SHIFTED or LBM_SC_FP32_SHIFTED_MATH64");
    if (c->packed_rows != 0 && c->packed_rows != 1) return fail(LBM_SC_EINVAL, "packed_rows must be 0 or 1");
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return fail(LBM_SC_EINVAL, "tau must be > 0.5");
    if (!std::isfinite(c->g_over_gc)) return fail(LBM_SC_EINVAL, "g_over_gc must be finite");
    if (c->geom != LBM_SC_FROM_HOST) {
        if (!(c->width > 0.0)) return fail(LBM_SC_EINVAL, "width must be > 0");
        if (c->geom == LBM_SC_SLAB) {
            if (c->slab_axis < 0 || c->slab_axis > 2) return fail(LBM_SC_EINVAL, "slab_axis must be 0..2");
            if (!(c->slab_thickness > 0.0)) return fail(LBM_SC_EINVAL, "slab_thickness must be > 0");
        } else if (!(c->radius > 0.0)) {
            return fail(LBM_SC_EINVAL, "radius must be > 0");
        }
        const bool auto_dens = c->n_in == 0.0 && c->n_out == 0.0;
        if (auto_dens && !(c->g_over_gc > 1.0))
            return fail(LBM_SC_EINVAL, "g_over_gc must be > 1 when the coexistence densities are computed");
        if (!auto_dens && !(c->n_in > 0.0 && c->n_out > 0.0))
            return fail(LBM_SC_EINVAL, "n_in and n_out must both be > 0 (or both 0)");
        if (!(c->noise_amp >= 0.0)) return fail(LBM_SC_EINVAL, "noise_amp must be >= 0");
    }
    if (!(c->rho_ref >= 0.0) || !std::isfinite(c->rho_ref)) return fail(LBM_SC_EINVAL, "rho_ref must be >= 0");
    // the step kernel addresses the 19 populations of one z-plane through one buffer resource of
    // at most 4 GiB
    const size_t elem = c->prec == LBM_SC_FP64 ? 8 : 4;
    const unsigned long long pxy = (unsigned long long)row_pitch(c->nx, elem, c->packed_rows) * c->ny;
    if (19ull * population_pitch(pxy, elem) * elem >= (1ull << 32))
        return fail(LBM_SC_EINVAL, "box too large: the 19 populations of one z-plane must fit in 4 GiB");
    return LBM_SC_OK;
}

void drop_box_graph(lbm_sc* h)
{
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    h->graph_len = 0;
}

// LBM_SC_EINVAL while the caller is capturing the stream: the calls guarded by this wait for the
// stream or copy through host memory, neither of which a capture can hold (inside a capture they
// would fail and end the caller's capture)
int refuse_in_capture(hipStream_t s, const char* what)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(LBM_SC_EINVAL, std::string(what) + " is not for use inside a stream capture");
    return LBM_SC_OK;
}

// Observation workspace, shared by the boxes of one device: density, psi and momentum of every
// node (5 doubles per node) while an observation (or a get/set staging copy, or the initial
// state) is computed. Every user holds the device's lock from the first launch that touches the
// workspace until its stream has drained, so the work of two boxes never overlaps in it. It grows
// to the largest box used and is freed when the last box of the device is destroyed. Only the
// previous observation's velocity (3 doubles per node) stays with each box.
struct Workspace {
    std::mutex mu;
    double* ptr = nullptr;
    size_t nodes = 0;    // capacity in nodes
    int boxes = 0;       // live boxes of the device
};
constexpr int MAX_DEVICES = 64;
Workspace g_ws[MAX_DEVICES];

// Make the (locked) workspace w of device dev hold n nodes: dn (n), dpsi (n), dj (3n).
int ws_reserve(Workspace& w, int dev, size_t n)
{
    if (w.nodes >= n) return LBM_SC_OK;
    int cur = dev;
    if (hipGetDevice(&cur) != hipSuccess) cur = dev;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_SC_EDEVICE, "hipSetDevice for the observation workspace failed");
    }
    if (w.ptr) (void)hipFree(w.ptr);   // its previous users have drained their streams
    w.ptr = nullptr;
    w.nodes = 0;
    hipError_t e = hipMalloc((void**)&w.ptr, 5 * n * sizeof(double));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        w.ptr = nullptr;
        (void)hipGetLastError();
        return fail(LBM_SC_ENOMEM, "observation workspace of " + std::to_string(5 * n * 8) +
                                       " bytes: " + hipGetErrorString(e));
    }
    w.nodes = n;
    return LBM_SC_OK;
}

void release(lbm_sc* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_box_graph(h);
    if (h->own_pop) {
        for (void* p : h->pop)
            if (p) (void)hipFree(p);
    }
    void* bufs[] = {h->d_uprev, h->d_parts, h->d_small, h->d_prof};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    {
        Workspace& w = g_ws[h->dev];
        std::lock_guard<std::mutex> lock(w.mu);
        if (--w.boxes == 0 && w.ptr) {
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.nodes = 0;
        }
    }
    delete h;
}

int alloc(lbm_sc* h, void** p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(LBM_SC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                       hipGetErrorString(e));
    }
    h->device_bytes += (int64_t)bytes;
    return LBM_SC_OK;
}

int profile_len(const lbm_sc* h)
{
    if (h->cfg.geom == LBM_SC_SLAB)
        return h->cfg.slab_axis == 0 ? h->box.nx : (h->cfg.slab_axis == 1 ? h->box.ny : h->box.nz);
    return h->box.nx;
}

// Run the observation kernels and assemble lbm_sc_obs on the host (synchronises). The caller
// holds the lock of the box's device workspace.
int observe(lbm_sc* h, lbm_sc_obs* o, double* prof_out)
{
    const lbm::BoxDesc& b = h->box;
    Workspace& w = g_ws[h->dev];
    if (int rc = ws_reserve(w, h->dev, b.n)) return rc;
    double* dn = w.ptr;
    double* dpsi = w.ptr + b.n;
    double* dj = w.ptr + 2 * (size_t)b.n;
    hipError_t le = lbm::launch_observe(h->fp32, b, h->pop[h->cur], dn, dpsi, dj, h->d_uprev,
                                        h->has_prev, h->d_parts, h->d_small, h->stream);
    const int L = profile_len(h);
    if (le == hipSuccess) {
        if (h->cfg.geom == LBM_SC_SLAB)
            le = lbm::launch_profile_planes(b, h->cfg.slab_axis, dn, dpsi, h->d_prof,
                                            h->d_small + lbm::OBS_PARTS, h->stream);
        else
            le = lbm::launch_profile_line(b, dn, dpsi, h->d_prof, h->d_small + lbm::OBS_PARTS,
                                          h->stream);
    }
    if (le != hipSuccess) {
        // nothing may still use the workspace once the lock is released
        (void)hipStreamSynchronize(h->stream);
        return fail_hip("observation launch", le);
    }
    double small[lbm::OBS_PARTS + 4];
    std::vector<double> prof(4 * (size_t)L);
    hipError_t e = hipMemcpyAsync(small, h->d_small, sizeof(small), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(prof.data(), h->d_prof, prof.size() * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream);
    // wait also when an enqueue failed: no copy may still write into small or prof after return
    const hipError_t se = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail_hip("hipMemcpyAsync", e);
    if (se != hipSuccess) return fail_hip("hipStreamSynchronize", se);

    std::memset(o, 0, sizeof(*o));
    const double nan = std::nan("");
    o->step = h->step;
    o->mass = small[0];
    o->mass0 = h->mass0;
    for (int c = 0; c < 3; ++c) o->mom[c] = small[1 + c];
    const int dims[3] = {b.nx, b.ny, b.nz};
    for (int c = 0; c < 3; ++c) o->com[c] = dims[c] / 2 + small[4 + c] / small[0];
    o->du_l1 = h->has_prev ? small[7] / (double)b.n : nan;
    o->du_max = h->has_prev ? small[8] : nan;
    o->has_du = h->has_prev;
    o->finite = small[9] == 0.0 ? 1 : 0;
    o->n_min = small[10];
    o->n_max = small[11];
    const double* probes = small + lbm::OBS_PARTS;
    o->n_center = probes[0];
    o->P_in = probes[1];
    o->n_far = probes[2];
    o->P_out = probes[3];
    o->dP = o->P_in - o->P_out;
    o->C = nan;
    o->R_s = nan;
    o->sigma_s = nan;
    o->R_e = nan;
    o->sigma0_flat = nan;
    o->pn_spread = nan;
    if (h->cfg.geom == LBM_SC_SLAB) {
        const int a = h->cfg.slab_axis, t = (a + 1) % 3;
        const double* PN = prof.data() + (size_t)(1 + a) * L;
        const double* PT = prof.data() + (size_t)(1 + t) * L;
        double s = 0.0, mx = PN[0], mn = PN[0];
        for (int k = L / 2; k < L; ++k) s += PN[k] - PT[k];
        for (int k = 0; k < L; ++k) {
            mx = std::fmax(mx, PN[k]);
            mn = std::fmin(mn, PN[k]);
        }
        o->sigma0_flat = s;
        o->pn_spread = mx - mn;
    } else {
        // C = int_0^{R_out} r^2 (P_out - P_T(r)) dr along +x from the centre, P_T = P^yy
        const int cx = b.nx / 2, R_out = b.nx - 1 - cx;
        const double* Pyy = prof.data() + 2 * (size_t)L;
        double C = 0.0;
        for (int r = 0; r < R_out; ++r) {
            const double y0 = (double)r * r * (o->P_out - Pyy[cx + r]);
            const double y1 = (double)(r + 1) * (r + 1) * (o->P_out - Pyy[cx + r + 1]);
            C += 0.5 * (y0 + y1);
        }
        o->C = C;
        if (o->dP > 0.0 && C > 0.0) {
            o->R_s = std::cbrt(6.0 * C / o->dP);
            o->sigma_s = 0.5 * o->dP * o->R_s;
        }
        const double V = (double)b.n;
        const double v = 3.0 * (o->mass - V * o->n_far) / (4.0 * M_PI * (o->n_center - o->n_far));
        o->R_e = std::cbrt(v);
    }
    if (prof_out) std::memcpy(prof_out, prof.data(), prof.size() * sizeof(double));
    h->has_prev = 1;
    return LBM_SC_OK;
}

// Tile width and height of a launch shape on a box (full-row tiles: the box's nx and the rows
// that fit; by < 1 means the box's rows are too long for them).
void tile_dims(const lbm::StepShape& s, const lbm::BoxDesc& b, int& bx, int& by)
{
    if (s.tile_x == 0) {
        bx = b.nx;
        by = lbm::row_tile_rows(s, b.px);
    } else {
        bx = s.tile_x;
        by = lbm::tile_height(s);
    }
}

bool shape_fits(const lbm::StepShape& s, const lbm::BoxDesc& b)
{
    int bx, by;
    tile_dims(s, b, bx, by);
    return bx >= 1 && by >= 1;
}

// Default launch shape (the fastest compiled shape measured on MI355X at 256^3). Single-precision
// arithmetic: 8-wave workgroups with two rows per wave (64 x 16 tiles), no prefetch (under 128
// VGPRs: two workgroups fit per CU). Double-precision arithmetic needs about twice the
// registers: FP32 storage with FP64 arithmetic takes 4-wave workgroups, 64 x 8 tiles, no
// prefetch, two workgroups per CU; FP64 storage takes 4-wave workgroups, 32 x 16 tiles, with the
// next plane prefetched (one workgroup per CU). XCD remap on. The z chunk minimises (rounds of
// workgroups over the resident slots) x (planes per chunk + the two planes each chunk pulls
// again): the slots draw the full bandwidth, so a partly filled last round costs a whole round
// (288 workgroups of a 192^3 box run 30 % slower than 252).
// z chunk of a launch with bx x by tiles and `slots` resident workgroups, each chunk pulling
// `extra` planes besides its own: minimises (rounds of workgroups over the slots) x (planes per
// chunk + extra), since the slots draw the full bandwidth and a partly filled last round costs a
// whole round.
int z_chunk_for(const lbm::BoxDesc& b, int bx, int by, int slots, int extra)
{
    const long tiles = (long)((b.nx + bx - 1) / bx) * ((b.ny + by - 1) / by);
    int best = b.nz;
    double best_cost = 0.0;
    for (int zc = 1; zc <= b.nz; ++zc) {
        const long chunks = (b.nz + zc - 1) / zc;
        if (zc > 1 && (b.nz + zc - 2) / (zc - 1) == chunks) continue;   // same split
        const long wgs = tiles * chunks;
        const double cost = (double)((wgs + slots - 1) / slots) * (zc + extra);
        if (zc == 1 || cost < best_cost) {
            best = zc;
            best_cost = cost;
        }
    }
    return best;
}

void default_shape(lbm_sc* h)
{
    h->shape.xcd_remap = 1;
    h->shape.tile_x = 64;
    h->shape.rows = 2;
    if (h->fp32 && !h->math64) {
        h->shape.waves = 8;
        h->shape.prefetch = 0;
    } else if (h->fp32) {
        h->shape.waves = 4;
        h->shape.prefetch = 0;
    } else {
        h->shape.waves = 4;
        h->shape.prefetch = 1;
        h->shape.tile_x = 32;
    }
    int cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    // without prefetch a CU needs eight resident waves (two workgroups of four) to cover the load
    // latency; with prefetch, or eight waves in one workgroup, one workgroup per CU suffices
    const int slots = cus * (h->shape.prefetch ? 1 : std::max(1, 8 / h->shape.waves));
    h->shape.z_chunk = z_chunk_for(h->box, h->shape.tile_x, lbm::tile_height(h->shape), slots, 2);
    // FP32 storage and arithmetic at tau = 1: two steps per pass, each chunk pulling 6 planes more
    // than it steps. Boxes of 2.3 M nodes or more: 32 x 16 tiles of 4 waves without prefetch (two
    // nodes per thread, 78 KB of LDS and 215 VGPRs without spills: two workgroups per CU);
    // smaller ones: 64 x 8 tiles of 8 waves with the next plane prefetched (one workgroup per CU).
    // Measured against the 64 x 8 tiles: 6 % faster at 136^3, 16 % at 144^3, 11-16 % from 160^3
    // to 384^3 (and 2-8 % faster than 32 x 16 tiles of 8 waves, whose 128 VGPRs spill), equal at
    // 112^3, 1 % slower at 128^3, 35-39 % slower at 48^3 and 64^3
    const bool big = (double)h->box.n >= 2.3e6;
    h->shape2.rows = big ? 2 : 1;
    h->shape2.waves = big ? 4 : 8;
    h->shape2.prefetch = big ? 0 : 1;
    h->shape2.tile_x = big ? 32 : 64;
    h->shape2.xcd_remap = 1;
    h->shape2.z_chunk = big ? z_chunk_for(h->box, 32, 16, 2 * cus, 6) : z_chunk_for(h->box, 64, 8, cus, 6);
    h->spp = (h->fp32 && !h->math64 && h->box.tau == 1.0) ? 2 : 1;
}

// What one box holds itself; the observation workspace (5 doubles per node) is shared per device.
struct Sizes {
    size_t popbytes, n24, parts, small, prof;
    size_t total() const { return 2 * popbytes + n24 + parts + small + prof; }
};

Sizes sizes_for(const lbm_sc_config* c)
{
    const size_t elem = c->prec == LBM_SC_FP64 ? 8 : 4;
    const unsigned long long n = (unsigned long long)c->nx * c->ny * c->nz;
    const unsigned long long pxy = (unsigned long long)row_pitch(c->nx, elem, c->packed_rows) * c->ny;
    const int Lmax = std::max(c->nx, std::max(c->ny, c->nz));
    Sizes s;
    s.popbytes = (size_t)c->nz * 19 * population_pitch(pxy, elem) * elem;
    s.n24 = 3 * (size_t)n * 8;
    s.parts = (size_t)lbm::OBS_BLOCKS * lbm::OBS_PARTS * 8;
    s.small = (lbm::OBS_PARTS + 4 + 1) * 8;   // scalars, probes, the two dither step counts
    s.prof = 4 * (size_t)Lmax * 8;
    return s;
}

}  // namespace

extern "C" {

const char* lbm_sc_last_error(void) { return g_err; }

int64_t lbm_sc_device_bytes(const lbm_sc_config* cfg)
{
    int rc = validate(cfg);
    if (rc) return rc;
    return (int64_t)sizes_for(cfg).total();
}

int64_t lbm_sc_population_bytes(const lbm_sc_config* cfg)
{
    int rc = validate(cfg);
    if (rc) return rc;
    return (int64_t)sizes_for(cfg).popbytes;
}

double lbm_sc_gc(int32_t psi)
{
    if (psi != LBM_SC_PSI_EXP && psi != LBM_SC_PSI_ONEMINUS) return std::nan("");
    return gc_h(psi);
}

int lbm_sc_coexistence(int32_t psi, double g_over_gc, double* n_gas, double* n_liquid, double* p0)
{
    if (psi != LBM_SC_PSI_EXP && psi != LBM_SC_PSI_ONEMINUS) return fail(LBM_SC_EINVAL, "unknown psi");
    if (!(g_over_gc > 1.0)) return fail(LBM_SC_EINVAL, "g_over_gc must be > 1");
    Coex c;
    if (!coexistence(psi, g_over_gc, c)) return fail(LBM_SC_EINVAL, "no flat coexistence found");
    if (n_gas) *n_gas = c.ng;
    if (n_liquid) *n_liquid = c.nl;
    if (p0) *p0 = c.p0;
    return LBM_SC_OK;
}

}  // extern "C"

namespace {

// A caller's population buffer: device memory of the current device, 256-byte aligned, with at
// least `need` bytes from p inside one allocation.
// LBM_SC_EINVAL unless [p, p + need) lies inside one device allocation of the current device.
int check_device_range(const void* p, size_t need, const std::string& name)
{
    hipPointerAttribute_t attr;
    int dev = -1;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_SC_EINVAL, std::string(name) + " is not device memory known to HIP");
    }
    if (attr.type != hipMemoryTypeDevice || attr.device != dev)
        return fail(LBM_SC_EINVAL, std::string(name) + " is not device memory of the current device");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_SC_EINVAL, std::string(name) + ": allocation range unknown");
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
    if (q < b || q - b + need > size)
        return fail(LBM_SC_EINVAL, std::string(name) + " has fewer than " + std::to_string(need) +
                                       " bytes in its allocation");
    return LBM_SC_OK;
}

int check_caller_buffer(const void* p, size_t need, const char* name)
{
    if (!p) return fail(LBM_SC_EINVAL, std::string(name) + " is NULL");
    if (reinterpret_cast<uintptr_t>(p) % 256 != 0)
        return fail(LBM_SC_EINVAL, std::string(name) + " is not 256-byte aligned");
    return check_device_range(p, need, name);
}

int create_box(const lbm_sc_config* cfg, void* buf_a, void* buf_b, size_t buf_bytes, lbm_sc** out)
{
    if (!out) return fail(LBM_SC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return fail(LBM_SC_EDEVICE, "no usable current HIP device");
    }
    lbm_sc* h = new (std::nothrow) lbm_sc();
    if (!h) return fail(LBM_SC_ENOMEM, "host allocation failed");
    h->dev = dev;
    {
        Workspace& w = g_ws[dev];
        std::lock_guard<std::mutex> lock(w.mu);
        ++w.boxes;   // from here release() accounts for the box
    }
    h->cfg = *cfg;
    h->fp32 = cfg->prec != LBM_SC_FP64;
    h->math64 = cfg->prec == LBM_SC_FP32_SHIFTED_MATH64;
    h->elem = h->fp32 ? 4 : 8;
    h->Gc = gc_h(cfg->psi);
    h->G = cfg->g_over_gc * h->Gc;

    double n_in = cfg->n_in, n_out = cfg->n_out;
    if (cfg->geom != LBM_SC_FROM_HOST && n_in == 0.0 && n_out == 0.0) {
        Coex c;
        if (!coexistence(cfg->psi, cfg->g_over_gc, c)) {
            release(h);
            return fail(LBM_SC_EINVAL, "no flat coexistence for this psi and g_over_gc");
        }
        n_in = cfg->geom == LBM_SC_BUBBLE ? c.ng : c.nl;
        n_out = cfg->geom == LBM_SC_BUBBLE ? c.nl : c.ng;
    }
    h->cfg.n_in = n_in;
    h->cfg.n_out = n_out;
    double rho_ref = 0.0;
    if (h->fp32) rho_ref = cfg->rho_ref > 0.0 ? cfg->rho_ref : 0.5 * (n_in + n_out);
    if (h->fp32 && !(rho_ref > 0.0)) {
        release(h);
        return fail(LBM_SC_EINVAL, "shifted FP32 storage with geom FROM_HOST needs rho_ref > 0");
    }
    h->cfg.rho_ref = rho_ref;

    lbm::BoxDesc& b = h->box;
    b.nx = cfg->nx;
    b.ny = cfg->ny;
    b.nz = cfg->nz;
    b.nxy = (unsigned)cfg->nx * (unsigned)cfg->ny;
    b.n = b.nxy * (unsigned)cfg->nz;
    b.px = row_pitch(cfg->nx, h->elem, cfg->packed_rows);
    const unsigned long long pxy = (unsigned long long)b.px * (unsigned)cfg->ny;
    b.pxy = (unsigned)pxy;   // < 2^32: validate bounds the plane
    b.pp = (unsigned)population_pitch(pxy, h->elem);   // 19 * pp * elem < 2^32 (validate)
    b.psi = cfg->psi;
    b.G = h->G;
    b.tau = cfg->tau;
    b.rho_ref = rho_ref;
    default_shape(h);

    if (cfg->stream) {
        h->stream = (hipStream_t)cfg->stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            h->stream = nullptr;
            release(h);
            return fail_hip("hipStreamCreateWithFlags", e);
        }
        h->own_stream = true;
    }

    const Sizes sz = sizes_for(cfg);
    if (buf_a || buf_b) {
        // caller-owned population buffers, used in place and never freed here
        const uintptr_t qa = reinterpret_cast<uintptr_t>(buf_a), qb = reinterpret_cast<uintptr_t>(buf_b);
        if (buf_bytes < sz.popbytes)
            rc = fail(LBM_SC_EINVAL, "bytes must be at least lbm_sc_population_bytes(cfg) = " +
                                         std::to_string(sz.popbytes));
        else if ((rc = check_caller_buffer(buf_a, sz.popbytes, "buffer a")) ||
                 (rc = check_caller_buffer(buf_b, sz.popbytes, "buffer b"))) {
        } else if (qa < qb + sz.popbytes && qb < qa + sz.popbytes) {
            rc = fail(LBM_SC_EINVAL, "buffers a and b overlap");
        }
        if (rc) {
            std::string msg = g_err;
            release(h);
            return fail(rc, msg);
        }
        h->own_pop = false;
        h->pop[0] = buf_a;
        h->pop[1] = buf_b;
    } else if ((rc = alloc(h, &h->pop[0], sz.popbytes)) || (rc = alloc(h, &h->pop[1], sz.popbytes))) {
        std::string msg = g_err;
        release(h);
        return fail(rc, msg);
    }
    if ((rc = alloc(h, (void**)&h->d_uprev, sz.n24)) ||
        (rc = alloc(h, (void**)&h->d_parts, sz.parts)) ||
        (rc = alloc(h, (void**)&h->d_small, sz.small)) ||
        (rc = alloc(h, (void**)&h->d_prof, sz.prof))) {
        std::string msg = g_err;
        release(h);
        return fail(rc, msg);
    }
    const size_t popbytes = sz.popbytes;
    // the two step counts that seed the FP32 dither sit after the scalars and probes; the
    // initial state (buffer 0) is step 0
    b.tick = reinterpret_cast<unsigned*>(h->d_small + lbm::OBS_PARTS + 4);
    {
        hipError_t e = hipMemsetAsync(b.tick, 0, 2 * sizeof(unsigned), h->stream);
        if (e != hipSuccess) {
            release(h);
            return fail_hip("hipMemsetAsync", e);
        }
    }

    if (cfg->geom != LBM_SC_FROM_HOST) {
        lbm::InitDesc& d = h->init;
        d.geom = cfg->geom == LBM_SC_SLAB ? 2 : 0;
        d.slab_axis = cfg->slab_axis;
        d.radius = cfg->geom == LBM_SC_SLAB ? 0.5 * cfg->slab_thickness : cfg->radius;
        d.width = cfg->width;
        d.n_in = n_in;
        d.n_out = n_out;
        d.noise_amp = cfg->noise_amp;
        d.seed = cfg->seed;
        {
            Workspace& w = g_ws[h->dev];
            std::lock_guard<std::mutex> lock(w.mu);
            rc = ws_reserve(w, h->dev, b.n);
            if (!rc) {
                hipError_t e = lbm::launch_init(h->fp32, b, d, w.ptr, w.ptr + b.n, h->pop[0],
                                                h->stream);
                if (e != hipSuccess) {
                    (void)hipStreamSynchronize(h->stream);
                    rc = fail_hip("launch_init", e);
                }
            }
            lbm_sc_obs o;
            if (!rc) rc = observe(h, &o, nullptr);
            if (!rc) h->mass0 = o.mass;
        }
        if (rc) {
            std::string msg = g_err;
            release(h);
            return fail(rc, msg);
        }
    } else {
        hipError_t e = hipMemsetAsync(h->pop[0], 0, popbytes, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            release(h);
            return fail_hip("hipMemsetAsync", e);
        }
    }
    h->cur = 0;
    h->step = 0;
    *out = h;
    return LBM_SC_OK;
}

}  // namespace

extern "C" {

int lbm_sc_create(const lbm_sc_config* cfg, lbm_sc** out)
{
    return create_box(cfg, nullptr, nullptr, 0, out);
}

int lbm_sc_create_with_buffers(const lbm_sc_config* cfg, void* a, void* b, size_t bytes, lbm_sc** out)
{
    if (!a || !b) {
        if (out) *out = nullptr;
        return fail(LBM_SC_EINVAL, "buffers a and b must both be given");
    }
    return create_box(cfg, a, b, bytes, out);
}

int lbm_sc_step(lbm_sc* h, int64_t nsteps)
{
    if (!h) return fail(LBM_SC_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(LBM_SC_EINVAL, "nsteps must be >= 0");
    // one launch advances the state by 1 or (two steps per pass) 2 time steps and moves it to the
    // other buffer
    auto launch = [&](int c, int steps) -> hipError_t {
        if (steps == 2)
            return lbm::launch_step2_f32(h->box, h->shape2, c, h->pop[c], h->pop[1 - c], h->stream);
        return lbm::launch_step(h->fp32, h->math64, h->box, h->shape, c, h->pop[c], h->pop[1 - c],
                                h->stream);
    };
    const int K = h->graph_steps;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(h->stream, &cs));
    // inside a caller's capture the launches are recorded into the caller's graph instead; each
    // recorded launch has fixed source and destination buffers, so only an even number of
    // launches leaves the state where a replay expects it (an odd one would recompute the same
    // step on every replay)
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (capturing && (nsteps & 1))
        return fail(LBM_SC_EINVAL, "inside a stream capture nsteps must be even");
    // two steps per pass: whole pairs of steps, and an even number of launches per graph or
    // caller capture; the rest (an odd last step, or a capture of 4k + 2 steps) goes one step
    // per launch
    const int spp = (h->spp == 2 && !(capturing && nsteps % 4)) ? 2 : 1;
    const int Kl = spp == 2 ? (K % 4 ? 0 : K / 2) : K;   // launches per graph
    const bool use_graph = Kl > 0 && nsteps >= K && !capturing;
    if (use_graph && (!h->graph || h->graph_len != K)) {
        // Kl (even) launches alternating the two buffers, starting from the current one
        drop_box_graph(h);
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        const int c = h->cur;
        hipError_t le = hipSuccess;
        for (int k = 0; k < Kl && le == hipSuccess; ++k) le = launch((c + k) & 1, spp);
        hipError_t ce = hipStreamEndCapture(h->stream, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail_hip("launch_step during capture", le);
        }
        if (ce != hipSuccess) return fail_hip("hipStreamEndCapture", ce);
        hipError_t ie = hipGraphInstantiate(&h->graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            h->graph = nullptr;
            return fail_hip("hipGraphInstantiate", ie);
        }
        h->graph_len = K;
        h->graph_cur = c;
    }
    int64_t done = 0;
    while (done < nsteps) {
        if (use_graph && h->graph && h->cur == h->graph_cur && nsteps - done >= h->graph_len) {
            HIP_TRY(hipGraphLaunch(h->graph, h->stream));
            done += h->graph_len;          // an even number of launches: same current buffer
        } else {
            const int steps = (spp == 2 && nsteps - done >= 2) ? 2 : 1;
            hipError_t e = launch(h->cur, steps);
            if (e != hipSuccess) return fail_hip("launch_step", e);
            h->cur = 1 - h->cur;
            done += steps;
        }
    }
    h->step += nsteps;
    return LBM_SC_OK;
}

int lbm_sc_sync(lbm_sc* h)
{
    if (!h) return fail(LBM_SC_EINVAL, "handle is NULL");
    if (int rc = refuse_in_capture(h->stream, "lbm_sc_sync")) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_SC_OK;
}

int lbm_sc_observables(lbm_sc* h, lbm_sc_obs* out, double* prof, size_t prof_len)
{
    if (!h || !out) return fail(LBM_SC_EINVAL, "handle or out is NULL");
    if (prof && prof_len != 4 * (size_t)profile_len(h))
        return fail(LBM_SC_EINVAL, "prof_len must be 4 * " + std::to_string(profile_len(h)));
    if (int rc = refuse_in_capture(h->stream, "lbm_sc_observables")) return rc;
    Workspace& w = g_ws[h->dev];
    std::lock_guard<std::mutex> lock(w.mu);
    int rc = observe(h, out, prof);
    if (rc) return rc;
    if (!out->finite) return fail(LBM_SC_EUNSTABLE, "non-finite value or n <= 0 in the state");
    return LBM_SC_OK;
}

int lbm_sc_get_populations(lbm_sc* h, double* f, size_t len)
{
    if (!h || !f) return fail(LBM_SC_EINVAL, "handle or f is NULL");
    const size_t N = h->box.n;
    if (len != 19 * N) return fail(LBM_SC_EINVAL, "len must be 19*nx*ny*nz");
    if (int rc = refuse_in_capture(h->stream, "lbm_sc_get_populations")) return rc;
    Workspace& w = g_ws[h->dev];
    std::lock_guard<std::mutex> lock(w.mu);
    if (int rc = ws_reserve(w, h->dev, N)) return rc;
    for (int i = 0; i < 19; ++i) {
        hipError_t e = lbm::launch_get(h->fp32, h->box, i, h->pop[h->cur], w.ptr, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(f + (size_t)i * N, w.ptr, N * 8, hipMemcpyDeviceToHost, h->stream);
        // wait also when an enqueue failed: the workspace is free again once the lock is released
        const hipError_t se = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail_hip("population read-back", e);
        if (se != hipSuccess) return fail_hip("hipStreamSynchronize", se);
    }
    return LBM_SC_OK;
}

int lbm_sc_set_populations(lbm_sc* h, const double* f, size_t len)
{
    if (!h || !f) return fail(LBM_SC_EINVAL, "handle or f is NULL");
    const size_t N = h->box.n;
    if (len != 19 * N) return fail(LBM_SC_EINVAL, "len must be 19*nx*ny*nz");
    if (int rc = refuse_in_capture(h->stream, "lbm_sc_set_populations")) return rc;
    // a set state starts again at step 0 (the dither sequence restarts with it)
    HIP_TRY(hipMemsetAsync(h->box.tick, 0, 2 * sizeof(unsigned), h->stream));
    Workspace& w = g_ws[h->dev];
    std::lock_guard<std::mutex> lock(w.mu);
    if (int rc = ws_reserve(w, h->dev, N)) return rc;
    for (int i = 0; i < 19; ++i) {
        hipError_t e = hipMemcpyAsync(w.ptr, f + (size_t)i * N, N * 8, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = lbm::launch_set(h->fp32, h->box, i, w.ptr, h->pop[h->cur], h->stream);
        // wait also when an enqueue failed: the copy must be done with f, and the workspace free,
        // before returning
        const hipError_t se = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail_hip("population upload", e);
        if (se != hipSuccess) return fail_hip("hipStreamSynchronize", se);
    }
    h->step = 0;
    h->has_prev = 0;
    lbm_sc_obs o;
    int rc = observe(h, &o, nullptr);
    if (rc) return rc;
    h->mass0 = o.mass;
    return LBM_SC_OK;
}

int lbm_sc_set_step(lbm_sc* h, int64_t step)
{
    if (!h) return fail(LBM_SC_EINVAL, "handle is NULL");
    if (step < 0) return fail(LBM_SC_EINVAL, "step must be >= 0");
    if (int rc = refuse_in_capture(h->stream, "lbm_sc_set_step")) return rc;
    // the dither's step count of the current buffer (kept modulo 2^32) follows the step counter
    const unsigned t = (unsigned)(uint64_t)step;
    HIP_TRY(hipMemcpyAsync(h->box.tick + h->cur, &t, sizeof(t), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->step = step;
    return LBM_SC_OK;
}

int lbm_sc_get_info(lbm_sc* h, lbm_sc_info* out)
{
    if (!h || !out) return fail(LBM_SC_EINVAL, "handle or out is NULL");
    std::memset(out, 0, sizeof(*out));
    out->G = h->G;
    out->Gc = h->Gc;
    out->n_in = h->cfg.n_in;
    out->n_out = h->cfg.n_out;
    out->rho_ref = h->cfg.rho_ref;
    out->nodes = (int64_t)h->box.n;
    out->device_bytes = h->device_bytes;
    out->bytes_per_step = (int64_t)2 * 19 * (int64_t)h->elem * (int64_t)h->box.n;
    int bx, by;
    if (h->spp == 2) {
        bx = h->shape2.tile_x;
        by = 8 * h->shape2.rows;
    } else {
        tile_dims(h->shape, h->box, bx, by);
    }
    out->block_x = bx;
    out->block_y = by;
    out->z_chunk = h->spp == 2 ? h->shape2.z_chunk : h->shape.z_chunk;
    return LBM_SC_OK;
}

int lbm_sc_set_launch(lbm_sc* h, const lbm_sc_launch* l)
{
    if (!h || !l) return fail(LBM_SC_EINVAL, "handle or launch is NULL");
    if (l->z_chunk < 1) return fail(LBM_SC_EINVAL, "z_chunk must be >= 1");
    if (l->xcd_remap != 0 && l->xcd_remap != 1) return fail(LBM_SC_EINVAL, "xcd_remap must be 0 or 1");
    if (l->prefetch != 0 && l->prefetch != 1) return fail(LBM_SC_EINVAL, "prefetch must be 0 or 1");
    if (l->graph_steps < 0 || l->graph_steps % 2 || l->graph_steps > 4096)
        return fail(LBM_SC_EINVAL, "graph_steps must be even, in [0, 4096]");
    if (l->steps_per_pass != 1 && l->steps_per_pass != 2)
        return fail(LBM_SC_EINVAL, "steps_per_pass must be 1 or 2");
    lbm::StepShape s;
    s.rows = l->rows;
    s.waves = l->waves;
    s.z_chunk = l->z_chunk < h->box.nz ? l->z_chunk : h->box.nz;
    s.xcd_remap = l->xcd_remap;
    s.prefetch = l->prefetch;
    s.tile_x = l->tile_x;
    if (l->steps_per_pass == 2) {
        if (!(h->fp32 && !h->math64 && h->box.tau == 1.0))
            return fail(LBM_SC_EINVAL, "two steps per pass need FP32 storage, FP32 arithmetic and tau = 1");
        if (!lbm::step2_shape_supported(s)) return fail(LBM_SC_EINVAL, SHAPE2_MSG);
        drop_box_graph(h);
        h->graph_steps = l->graph_steps;
        h->spp = 2;
        h->shape2 = s;
        return LBM_SC_OK;
    }
    if (!lbm::shape_supported(s))
        return fail(LBM_SC_EINVAL, SHAPE_MSG);
    if (!shape_fits(s, h->box))
        return fail(LBM_SC_EINVAL, "rows too long for full-row tiles of this size (use more nodes per "
                                   "thread or tile_x 64)");
    if (s.tile_x == 0 && s.rows == 8 && (!h->fp32 || h->math64))
        return fail(LBM_SC_EINVAL, "full-row tiles with 8 nodes per thread need FP32 arithmetic");
    drop_box_graph(h);
    h->graph_steps = l->graph_steps;
    h->spp = 1;
    h->shape = s;
    return LBM_SC_OK;
}

int lbm_sc_get_launch(lbm_sc* h, lbm_sc_launch* out)
{
    if (!h || !out) return fail(LBM_SC_EINVAL, "handle or out is NULL");
    const lbm::StepShape& s = h->spp == 2 ? h->shape2 : h->shape;
    out->rows = s.rows;
    out->z_chunk = s.z_chunk;
    out->xcd_remap = s.xcd_remap;
    out->prefetch = s.prefetch;
    out->waves = s.waves;
    out->tile_x = s.tile_x;
    out->graph_steps = h->graph_steps;
    out->steps_per_pass = h->spp;
    return LBM_SC_OK;
}

int lbm_sc_stream_copy(const void* src, void* dst, size_t bytes, int32_t lane_bytes, void* stream)
{
    if (!src || !dst) return fail(LBM_SC_EINVAL, "src or dst is NULL");
    if (lane_bytes != 4 && lane_bytes != 8 && lane_bytes != 16)
        return fail(LBM_SC_EINVAL, "lane_bytes must be 4, 8 or 16");
    if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return fail(LBM_SC_EINVAL, "bytes and both pointers must be multiples of 16");
    const char* s = (const char*)src;
    const char* d = (const char*)dst;
    if (s < d + bytes && d < s + bytes) return fail(LBM_SC_EINVAL, "src and dst overlap");
    if (int rc = check_device_range(src, bytes, "src")) return rc;
    if (int rc = check_device_range(dst, bytes, "dst")) return rc;
    HIP_TRY(lbm::launch_stream_copy(src, dst, bytes, lane_bytes, (hipStream_t)stream));
    return LBM_SC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Groups
// ------------------------------------------------------------------------------------------

struct lbm_sc_group {
    hipStream_t stream = nullptr;
    std::vector<lbm_sc*> boxes;
    std::vector<lbm::GroupBox> desc;
    lbm::GroupBox* d_desc = nullptr;
    size_t d_desc_cap = 0;
    lbm::QueueState* d_queue = nullptr;
    unsigned* d_order = nullptr;  // two steps per pass with XCD remap: item order, 8 runs of order_per
    size_t d_order_cap = 0;
    unsigned order_per = 0;
    bool use_order = false;
    lbm_sc_group_launch launch;
    bool fp32 = false;
    bool math64 = false;          // FP32 storage with FP64 arithmetic (shared by every box)
    unsigned nitems = 0;
    int64_t nodes = 0;
    int64_t bytes_per_step = 0;
    bool dirty = true;            // work list must be rebuilt and uploaded
    int par = 0;                  // steps since the last rebuild, mod 2 (kernel parity)
    hipGraphExec_t graph = nullptr;
    int graph_len = 0;
};

namespace {

void detach(lbm_sc* b, lbm_sc_group* g)
{
    b->groups.erase(std::remove(b->groups.begin(), b->groups.end(), g), b->groups.end());
}

void drop_graph(lbm_sc_group* g)
{
    if (g->graph) (void)hipGraphExecDestroy(g->graph);
    g->graph = nullptr;
    g->graph_len = 0;
}

lbm::StepShape group_shape(const lbm_sc_group_launch& L)
{
    lbm::StepShape s;
    s.rows = L.rows;
    s.waves = L.waves;
    s.z_chunk = L.z_chunk > 0 ? L.z_chunk : 1;   // 0: per-box chunks (in the work list)
    s.xcd_remap = L.xcd_remap;
    s.prefetch = L.prefetch;
    s.tile_x = L.tile_x;
    return s;
}

int group_spp(const lbm_sc_group_launch& L) { return L.steps_per_pass == 2 ? 2 : 1; }

// Tile width and height of the group's items on box b (two steps per pass: tile_x x 8 * rows).
void group_tile_dims(const lbm_sc_group_launch& L, const lbm::BoxDesc& b, int& bx, int& by)
{
    if (group_spp(L) == 2) {
        bx = L.tile_x;
        by = 8 * L.rows;
    } else {
        tile_dims(group_shape(L), b, bx, by);
    }
}

// Whether box h (the i-th of a list) can be stepped by launch L; fails with the reason if not.
int check_group_box(const lbm_sc_group_launch& L, const lbm_sc* h, int i)
{
    const std::string who = "box " + std::to_string(i);
    if (group_spp(L) == 2) {
        if (!(h->fp32 && !h->math64 && h->box.tau == 1.0))
            return fail(LBM_SC_EINVAL, who + ": two steps per pass need FP32 storage, FP32 arithmetic "
                                             "and tau = 1");
        return LBM_SC_OK;
    }
    if (!shape_fits(group_shape(L), h->box))
        return fail(LBM_SC_EINVAL, who + ": rows too long for the full-row tiles of this launch");
    if (L.tile_x == 0 && L.rows == 8 && (!h->fp32 || h->math64))
        return fail(LBM_SC_EINVAL, "full-row tiles with 8 nodes per thread need FP32 arithmetic");
    return LBM_SC_OK;
}

// z_chunk 0: each box is cut into z chunks of about the same work, items_per_cu items per CU in
// total, so that small boxes march their whole height (no chunk ends pulled twice) and large
// ones are split for balance. Returns the work (nodes) of one item, 0 for fixed z chunks.
double chunk_work(lbm_sc* const* boxes, size_t nbox, const lbm_sc_group_launch& L)
{
    if (L.z_chunk != 0) return 0.0;
    double total = 0.0;
    for (size_t i = 0; i < nbox; ++i) total += (double)boxes[i]->box.n;
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    const int per_cu = L.items_per_cu > 0 ? L.items_per_cu : 8;
    return total / ((double)per_cu * cus);
}

// Work-list descriptor of box h under launch L; its items start at item_begin.
lbm::GroupBox box_desc(const lbm_sc* h, const lbm_sc_group_launch& L, double item_work,
                       unsigned item_begin)
{
    const lbm::StepShape shape = group_shape(L);
    int bx, by;
    group_tile_dims(L, h->box, bx, by);
    lbm::GroupBox d;
    std::memset(&d, 0, sizeof(d));
    d.b = h->box;
    d.pop[0] = h->pop[0];
    d.pop[1] = h->pop[1];
    d.phase = h->cur;
    d.by = shape.tile_x == 0 ? by : 0;
    d.tiles_x = (h->box.nx + bx - 1) / bx;
    d.tiles_y = (h->box.ny + by - 1) / by;
    if (L.z_chunk == 0) {
        const double tiles = (double)d.tiles_x * d.tiles_y;
        long chunks = item_work > 0.0 ? std::lround((double)h->box.n / item_work / tiles) : 1;
        chunks = std::max(1L, std::min(chunks, (long)h->box.nz));
        d.zc = (int)((h->box.nz + chunks - 1) / chunks);
    } else {
        d.zc = L.z_chunk < h->box.nz ? L.z_chunk : h->box.nz;
    }
    const unsigned nch = (unsigned)((h->box.nz + d.zc - 1) / d.zc);
    d.item_begin = item_begin;
    d.items = (unsigned)d.tiles_x * (unsigned)d.tiles_y * nch;
    return d;
}

// Nodes updated by item `it` (0 <= it < d.items) of a box's descriptor.
double item_nodes(const lbm::GroupBox& d, const lbm_sc_group_launch& L, unsigned it)
{
    int bx, by;
    group_tile_dims(L, d.b, bx, by);
    const unsigned tix = it % d.tiles_x, t2 = it / d.tiles_x;
    const unsigned tiy = t2 % d.tiles_y, ch = t2 / d.tiles_y;
    const int w = std::min(bx, d.b.nx - (int)tix * bx);
    const int hgt = std::min(by, d.b.ny - (int)tiy * by);
    const int dz = std::min(d.zc, d.b.nz - (int)ch * d.zc);
    return (double)std::max(w, 1) * std::max(hgt, 1) * std::max(dz, 1);
}

// Queue state of the persistent kernel: eight contiguous, work-balanced runs of the box-major
// item list (desc(i) returns the descriptor of box i), counters at zero.
template <typename Desc>
lbm::QueueState queue_ranges(Desc desc, size_t nbox, unsigned nitems, const lbm_sc_group_launch& L)
{
    lbm::QueueState q;
    std::memset(&q, 0, sizeof(q));
    double total = 0.0;
    for (size_t i = 0; i < nbox; ++i) {
        const lbm::GroupBox d = desc(i);
        for (unsigned it = 0; it < d.items; ++it) total += item_nodes(d, L, it);
    }
    // walk the items in order; queue x starts at the first item whose midpoint lies past x/8 of
    // the total work
    size_t bi = 0;
    unsigned it = 0, k = 0;
    lbm::GroupBox cur = nbox ? desc(0) : lbm::GroupBox{};
    double acc = 0.0;
    q.range[0] = 0;
    for (int x = 1; x < 8; ++x) {
        const double target = total * x / 8.0;
        while (k < nitems) {
            while (it >= cur.items && bi + 1 < nbox) {
                cur = desc(++bi);
                it = 0;
            }
            const double w = item_nodes(cur, L, it);
            if (!(acc + 0.5 * w < target)) break;
            acc += w;
            ++it;
            ++k;
        }
        q.range[x] = k;
    }
    q.range[8] = nitems;
    return q;
}

// Item order of the two-steps-per-pass group kernel (workgroup w on XCD w mod 8 takes entry
// (w mod 8) * per + w / 8): the box-major list cut into 8 contiguous runs of about equal cost, one
// per XCD, each run with its longest items first, so that the XCDs finish together and the short
// items fill the end of the launch. The cost of an item is the number of planes its march
// iterates: its chunk height plus the 6 planes pulled beyond it. The sort is stable, so the tiles
// of one box and z chunk stay together (neighbours in x and y run side by side on one XCD and
// share their halo lines in its L2). Returns false if the result is not a permutation.
bool two_step_order(const std::vector<lbm::GroupBox>& desc, unsigned nitems, std::vector<unsigned>& order,
                    unsigned& per)
{
    std::vector<double> cost(nitems);
    double total = 0.0;
    for (const lbm::GroupBox& d : desc) {
        const unsigned tiles = (unsigned)d.tiles_x * (unsigned)d.tiles_y;
        for (unsigned it = 0; it < d.items; ++it) {
            const int ch = (int)(it / tiles);
            const int dz = std::min(d.zc, d.b.nz - ch * d.zc);
            cost[d.item_begin + it] = dz + 6.0;
            total += dz + 6.0;
        }
    }
    unsigned bounds[9];
    bounds[0] = 0;
    int x = 1;
    double acc = 0.0;
    for (unsigned k = 0; k < nitems && x < 8; ++k) {
        while (x < 8 && !(acc + 0.5 * cost[k] < total * x / 8.0)) bounds[x++] = k;
        acc += cost[k];
    }
    while (x < 8) bounds[x++] = nitems;
    bounds[8] = nitems;
    per = 1;
    for (int r = 0; r < 8; ++r) per = std::max(per, bounds[r + 1] - bounds[r]);
    order.assign((size_t)8 * per, lbm::NO_ITEM);
    std::vector<unsigned> run;
    for (int r = 0; r < 8; ++r) {
        run.clear();
        for (unsigned k = bounds[r]; k < bounds[r + 1]; ++k) run.push_back(k);
        std::stable_sort(run.begin(), run.end(), [&](unsigned a, unsigned b) { return cost[a] > cost[b]; });
        std::copy(run.begin(), run.end(), order.begin() + (size_t)r * per);
    }
    std::vector<char> seen(nitems, 0);
    unsigned count = 0;
    for (unsigned v : order) {
        if (v == lbm::NO_ITEM) continue;
        if (v >= nitems || seen[v]) return false;
        seen[v] = 1;
        ++count;
    }
    return count == nitems;
}

// Build the work list and queue ranges for the current boxes and launch shape, and upload them.
// Phases align every box's current buffer with parity 0.
int group_rebuild(lbm_sc_group* g)
{
    const lbm_sc_group_launch& L = g->launch;
    g->desc.clear();
    g->nitems = 0;
    g->nodes = 0;
    g->bytes_per_step = 0;
    const double item_work = chunk_work(g->boxes.data(), g->boxes.size(), L);
    for (lbm_sc* h : g->boxes) {
        const lbm::GroupBox d = box_desc(h, L, item_work, g->nitems);
        g->nitems += d.items;
        g->nodes += (int64_t)h->box.n;
        g->bytes_per_step += (int64_t)2 * 19 * (int64_t)h->elem * (int64_t)h->box.n;
        g->desc.push_back(d);
    }
    if (!g->desc.empty()) {
        const size_t bytes = g->desc.size() * sizeof(lbm::GroupBox);
        if (bytes > g->d_desc_cap) {
            if (g->d_desc) (void)hipFree(g->d_desc);
            g->d_desc = nullptr;
            g->d_desc_cap = 0;
            hipError_t e = hipMalloc((void**)&g->d_desc, bytes);
            if (e != hipSuccess) return fail(LBM_SC_ENOMEM, "group descriptor allocation failed");
            g->d_desc_cap = bytes;
        }
        HIP_TRY(hipMemcpyAsync(g->d_desc, g->desc.data(), bytes, hipMemcpyHostToDevice, g->stream));
    }
    const lbm::QueueState q = queue_ranges([&](size_t i) { return g->desc[i]; }, g->desc.size(),
                                           g->nitems, L);
    HIP_TRY(hipMemcpyAsync(g->d_queue, &q, sizeof(q), hipMemcpyHostToDevice, g->stream));
    std::vector<unsigned> order;
    g->use_order = group_spp(L) == 2 && L.xcd_remap && g->nitems > 0;
    if (g->use_order) {
        if (!two_step_order(g->desc, g->nitems, order, g->order_per))
            return fail(LBM_SC_EDEVICE, "internal error: the item order is not a permutation");
        const size_t bytes = order.size() * sizeof(unsigned);
        if (bytes > g->d_order_cap) {
            if (g->d_order) (void)hipFree(g->d_order);
            g->d_order = nullptr;
            g->d_order_cap = 0;
            hipError_t e = hipMalloc((void**)&g->d_order, bytes);
            if (e != hipSuccess) return fail(LBM_SC_ENOMEM, "group item order allocation failed");
            g->d_order_cap = bytes;
        }
        HIP_TRY(hipMemcpyAsync(g->d_order, order.data(), bytes, hipMemcpyHostToDevice, g->stream));
    }
    // the queue state and the order are read by later launches: keep the host copies alive until
    // they have landed
    HIP_TRY(hipStreamSynchronize(g->stream));
    drop_graph(g);
    g->dirty = false;
    g->par = 0;
    return LBM_SC_OK;
}

hipError_t group_launch(lbm_sc_group* g, int parity)
{
    const lbm::StepShape s = group_shape(g->launch);
    if (group_spp(g->launch) == 2)
        return lbm::launch_group2_f32(s, g->d_desc, (int)g->desc.size(), g->nitems,
                                      g->use_order ? g->d_order : nullptr, g->order_per, parity,
                                      g->stream);
    const unsigned workers = g->launch.workers ? (unsigned)g->launch.workers : 256u;
    return lbm::launch_step_group(g->fp32, g->math64, s, g->d_desc, (int)g->desc.size(), g->nitems, parity,
                                  g->launch.persistent, workers, g->d_queue, g->stream);
}

int check_group_launch(const lbm_sc_group_launch* l)
{
    if (l->z_chunk < 0) return fail(LBM_SC_EINVAL, "z_chunk must be >= 0 (0: per-box chunks)");
    if (l->items_per_cu < 0 || l->items_per_cu > 4096)
        return fail(LBM_SC_EINVAL, "items_per_cu must be in [0, 4096]");
    if ((l->xcd_remap | l->prefetch | l->persistent) & ~1) return fail(LBM_SC_EINVAL, "flags must be 0 or 1");
    if (l->steps_per_pass < 0 || l->steps_per_pass > 2)
        return fail(LBM_SC_EINVAL, "steps_per_pass must be 0, 1 or 2");
    if (l->steps_per_pass == 2) {
        if (!lbm::step2_shape_supported(group_shape(*l))) return fail(LBM_SC_EINVAL, SHAPE2_MSG);
        if (l->persistent) return fail(LBM_SC_EINVAL, "two steps per pass take one workgroup per item (persistent 0)");
    } else if (!lbm::shape_supported(group_shape(*l))) {
        return fail(LBM_SC_EINVAL, SHAPE_MSG);
    }
    if (l->workers < 0 || l->workers % 8 || l->workers > 65536)
        return fail(LBM_SC_EINVAL, "workers must be a multiple of 8 in [0, 65536]");
    if (l->graph_steps < 0 || l->graph_steps % 2 || l->graph_steps > 4096)
        return fail(LBM_SC_EINVAL, "graph_steps must be even, in [0, 4096]");
    return LBM_SC_OK;
}

}  // namespace

extern "C" {

int lbm_sc_group_create(void* stream, lbm_sc_group** out)
{
    if (!out) return fail(LBM_SC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!stream) return fail(LBM_SC_EINVAL, "a group needs an explicit stream");
    lbm_sc_group* g = new (std::nothrow) lbm_sc_group();
    if (!g) return fail(LBM_SC_ENOMEM, "host allocation failed");
    g->stream = (hipStream_t)stream;
    g->launch = {2, 32, 1, 1, 0, 0, 64, 4, 64, 0, 1};   // rows 2, z chunk 32, 4 waves, 64-wide
    hipError_t e = hipMalloc((void**)&g->d_queue, sizeof(lbm::QueueState));
    if (e != hipSuccess) {
        delete g;
        return fail(LBM_SC_ENOMEM, "queue allocation failed");
    }
    e = hipMemsetAsync(g->d_queue, 0, sizeof(lbm::QueueState), g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        (void)hipFree(g->d_queue);
        delete g;
        return fail_hip("hipMemsetAsync", e);
    }
    *out = g;
    return LBM_SC_OK;
}

int lbm_sc_group_set(lbm_sc_group* g, lbm_sc* const* boxes, int32_t nbox)
{
    if (!g) return fail(LBM_SC_EINVAL, "group is NULL");
    if (nbox < 0 || (nbox > 0 && !boxes)) return fail(LBM_SC_EINVAL, "bad box list");
    if (int rc = refuse_in_capture(g->stream, "lbm_sc_group_set")) return rc;
    for (int i = 0; i < nbox; ++i) {
        if (!boxes[i]) return fail(LBM_SC_EINVAL, "box " + std::to_string(i) + " is NULL");
        if (boxes[i]->stream != g->stream)
            return fail(LBM_SC_EINVAL, "box " + std::to_string(i) + " was not created on the group's stream");
        if (boxes[i]->fp32 != boxes[0]->fp32 || boxes[i]->math64 != boxes[0]->math64)
            return fail(LBM_SC_EINVAL, "all boxes of a group must share one precision");
        for (int j = 0; j < i; ++j)
            if (boxes[j] == boxes[i]) return fail(LBM_SC_EINVAL, "a box appears twice");
        if (int rc = check_group_box(g->launch, boxes[i], i)) return rc;
    }
    for (lbm_sc* b : g->boxes) detach(b, g);
    g->boxes.assign(boxes, boxes + nbox);
    for (lbm_sc* b : g->boxes) b->groups.push_back(g);
    g->fp32 = nbox > 0 && boxes[0]->fp32;
    g->math64 = nbox > 0 && boxes[0]->math64;
    return group_rebuild(g);
}

int lbm_sc_group_step(lbm_sc_group* g, int64_t nsteps)
{
    if (!g) return fail(LBM_SC_EINVAL, "group is NULL");
    if (nsteps < 0) return fail(LBM_SC_EINVAL, "nsteps must be >= 0");
    if (int rc = refuse_in_capture(g->stream, "lbm_sc_group_step")) return rc;
    if (g->boxes.empty() || nsteps == 0) return LBM_SC_OK;
    // a box stepped alone since the last call is out of phase with the work list: rebuild (so
    // does a work list that does not match the boxes, e.g. after a failed rebuild)
    if (g->desc.size() != g->boxes.size()) g->dirty = true;
    for (size_t i = 0; i < g->boxes.size() && !g->dirty; ++i)
        if (((g->desc[i].phase + g->par) & 1) != g->boxes[i]->cur) g->dirty = true;
    if (g->dirty) {
        int rc = group_rebuild(g);
        if (rc) return rc;
    }
    const int K = g->launch.graph_steps;
    // two steps per pass: a graph of K steps holds K / 2 launches, an even number only when K is
    // a multiple of 4 (otherwise plain launches)
    const int spp = group_spp(g->launch);
    const int Kl = spp == 2 ? (K % 4 ? 0 : K / 2) : K;
    if (Kl > 0 && nsteps >= K && (!g->graph || g->graph_len != K)) {
        // capture Kl launches with parities 0, 1, ..., replayed whenever the parity is 0
        drop_graph(g);
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        for (int k = 0; k < Kl && le == hipSuccess; ++k) le = group_launch(g, k & 1);
        hipError_t ce = hipStreamEndCapture(g->stream, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail_hip("group launch during capture", le);
        }
        if (ce != hipSuccess) return fail_hip("hipStreamEndCapture", ce);
        hipError_t ie = hipGraphInstantiate(&g->graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            g->graph = nullptr;
            return fail_hip("hipGraphInstantiate", ie);
        }
        g->graph_len = K;
    }
    int64_t done = 0;
    while (done < nsteps) {
        if (g->graph && g->par == 0 && nsteps - done >= g->graph_len) {
            HIP_TRY(hipGraphLaunch(g->graph, g->stream));
            done += g->graph_len;
        } else if (spp == 2 && nsteps - done == 1) {
            // odd last step of a two-steps-per-pass group: each box alone, in its own single-step
            // shape (same arithmetic, so the same bits); the phases stay aligned with the parity
            for (size_t i = 0; i < g->boxes.size(); ++i) {
                lbm_sc* h = g->boxes[i];
                const int c = (g->desc[i].phase + g->par) & 1;
                HIP_TRY(lbm::launch_step(h->fp32, h->math64, h->box, h->shape, c, h->pop[c],
                                         h->pop[1 - c], g->stream));
            }
            g->par ^= 1;
            ++done;
        } else {
            HIP_TRY(group_launch(g, g->par));
            g->par ^= 1;
            done += spp;
        }
    }
    for (size_t i = 0; i < g->boxes.size(); ++i) {
        lbm_sc* h = g->boxes[i];
        h->cur = (g->desc[i].phase + g->par) & 1;
        h->step += nsteps;
    }
    return LBM_SC_OK;
}

int lbm_sc_group_set_launch(lbm_sc_group* g, const lbm_sc_group_launch* l)
{
    if (!g || !l) return fail(LBM_SC_EINVAL, "group or launch is NULL");
    int rc = check_group_launch(l);
    if (rc) return rc;
    if ((rc = refuse_in_capture(g->stream, "lbm_sc_group_set_launch"))) return rc;
    for (size_t i = 0; i < g->boxes.size(); ++i)
        if (int rc = check_group_box(*l, g->boxes[i], (int)i)) return rc;
    g->launch = *l;
    return group_rebuild(g);
}

int lbm_sc_group_get_launch(lbm_sc_group* g, lbm_sc_group_launch* out)
{
    if (!g || !out) return fail(LBM_SC_EINVAL, "group or out is NULL");
    *out = g->launch;
    return LBM_SC_OK;
}

int lbm_sc_group_info(lbm_sc_group* g, int32_t* nbox, int64_t* items, int64_t* nodes,
                      int64_t* bytes_per_step)
{
    if (!g) return fail(LBM_SC_EINVAL, "group is NULL");
    if (g->dirty && !g->boxes.empty()) {   // a box left (destroyed): count the rebuilt work list
        if (int rc = refuse_in_capture(g->stream, "lbm_sc_group_info")) return rc;
        if (int rc = group_rebuild(g)) return rc;
    }
    if (nbox) *nbox = (int32_t)g->boxes.size();
    if (items) *items = g->nitems;
    if (nodes) *nodes = g->nodes;
    if (bytes_per_step) *bytes_per_step = g->bytes_per_step;
    return LBM_SC_OK;
}

void lbm_sc_group_destroy(lbm_sc_group* g)
{
    if (!g) return;
    for (lbm_sc* b : g->boxes) detach(b, g);
    (void)hipStreamSynchronize(g->stream);
    drop_graph(g);
    if (g->d_desc) (void)hipFree(g->d_desc);
    if (g->d_queue) (void)hipFree(g->d_queue);
    if (g->d_order) (void)hipFree(g->d_order);
    delete g;
}

int lbm_sc_step_boxes_noalloc(lbm_sc* const* boxes, int32_t nbox, int64_t nsteps,
                              const lbm_sc_group_launch* launch)
{
    if (nbox < 0 || (nbox > 0 && !boxes) || !launch) return fail(LBM_SC_EINVAL, "bad box list or launch");
    if (nbox > lbm::NOALLOC_MAX_BOXES)
        return fail(LBM_SC_EINVAL, "lbm_sc_step_boxes_noalloc takes at most 1024 boxes");
    if (nsteps < 0) return fail(LBM_SC_EINVAL, "nsteps must be >= 0");
    if (int rc = check_group_launch(launch)) return rc;
    const lbm_sc_group_launch& L = *launch;
    const lbm::StepShape shape = group_shape(L);
    for (int i = 0; i < nbox; ++i) {
        const lbm_sc* b = boxes[i];
        if (!b) return fail(LBM_SC_EINVAL, "a box is NULL");
        if (b->stream != boxes[0]->stream)
            return fail(LBM_SC_EINVAL, "all boxes must have been created on one stream");
        if (b->fp32 != boxes[0]->fp32 || b->math64 != boxes[0]->math64)
            return fail(LBM_SC_EINVAL, "all boxes must share one precision");
        for (int j = 0; j < i; ++j)
            if (boxes[j] == b) return fail(LBM_SC_EINVAL, "a box appears twice");
        if (int rc = check_group_box(L, b, i)) return rc;
    }
    if (nbox == 0 || nsteps == 0) return LBM_SC_OK;
    hipStream_t st = boxes[0]->stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    // a recorded launch has fixed source and destination buffers: only an even count leaves every
    // box where a replay expects it
    if (cs != hipStreamCaptureStatusNone && (nsteps & 1))
        return fail(LBM_SC_EINVAL, "inside a stream capture nsteps must be even");
    void* scratch = nullptr;
    HIP_TRY(lbm::noalloc_scratch_address(&scratch));

    // work list, written into the device array in batches carried by kernel arguments (no host
    // staging buffer, no device allocation); phases align every box's current buffer with parity 0
    const double item_work = chunk_work(boxes, (size_t)nbox, L);
    lbm::DescBatch batch;
    std::memset(&batch, 0, sizeof(batch));
    unsigned nitems = 0;
    for (int i = 0; i < nbox; ++i) {
        const lbm::GroupBox d = box_desc(boxes[i], L, item_work, nitems);
        if ((uint64_t)nitems + d.items > 0xFFFFFFFFull)
            return fail(LBM_SC_EINVAL, "too many work items");
        nitems += d.items;
        if (batch.count == 0) batch.first = i;
        batch.d[batch.count++] = d;
        if (batch.count == lbm::NOALLOC_BATCH || i == nbox - 1) {
            HIP_TRY(lbm::launch_put_descs(batch, scratch, st));
            batch.count = 0;
        }
    }
    const lbm::GroupBox* d_desc = static_cast<const lbm::GroupBox*>(scratch);
    lbm::QueueState* d_queue = reinterpret_cast<lbm::QueueState*>(static_cast<char*>(scratch) +
                                                                  lbm::noalloc_queue_offset());
    if (L.persistent) {
        // the queue ranges, with every counter at zero (the kernel's last workgroup clears them
        // again after each launch)
        const lbm::QueueState q = queue_ranges(
            [&](size_t i) { return box_desc(boxes[i], L, item_work, 0); }, (size_t)nbox, nitems, L);
        HIP_TRY(lbm::launch_put_queue(q, scratch, st));
    }
    const unsigned workers = L.workers ? (unsigned)L.workers : 256u;
    const bool fp32 = boxes[0]->fp32, math64 = boxes[0]->math64;
    // done: steps taken; flips: launches, each moving every box to its other buffer
    int64_t done = 0, flips = 0;
    hipError_t e = hipSuccess;
    if (group_spp(L) == 1) {
        for (; done < nsteps && e == hipSuccess; ++done, ++flips)
            e = lbm::launch_step_group(fp32, math64, shape, d_desc, nbox, nitems, (int)(flips & 1),
                                       L.persistent, workers, d_queue, st);
        if (e != hipSuccess) {   // the failed launch did not step
            --done;
            --flips;
        }
    } else {
        // two steps per launch (the items in list order: no per-XCD item order, which would not
        // fit the fixed array); the rest as single steps of each box alone in its own single-step
        // shape: an odd last step, and inside a caller's capture the last pair of a count of
        // 4k + 2, so that the recorded launches move every box an even number of times
        int64_t pairs = nsteps / 2;
        if (cs != hipStreamCaptureStatusNone && (pairs & 1)) --pairs;
        for (int64_t k = 0; k < pairs && e == hipSuccess; ++k) {
            e = lbm::launch_group2_f32(shape, d_desc, nbox, nitems, nullptr, 0, (int)(flips & 1), st);
            if (e == hipSuccess) {
                done += 2;
                ++flips;
            }
        }
        while (done < nsteps && e == hipSuccess) {
            for (int i = 0; i < nbox && e == hipSuccess; ++i) {
                const lbm_sc* h = boxes[i];
                const int c = (int)((h->cur + flips) & 1);
                e = lbm::launch_step(h->fp32, h->math64, h->box, h->shape, c, h->pop[c], h->pop[1 - c], st);
            }
            if (e == hipSuccess) {
                ++done;
                ++flips;
            }
        }
    }
    for (int i = 0; i < nbox; ++i) {
        lbm_sc* h = boxes[i];
        h->cur = (int)((h->cur + flips) & 1);
        h->step += done;
    }
    if (e != hipSuccess) return fail_hip("multi-box step launch", e);
    return LBM_SC_OK;
}

void lbm_sc_destroy(lbm_sc* h)
{
    if (!h) return;
    // leave every group that lists the box, so that no group launch reaches its freed buffers:
    // the group's next step rebuilds its work list without it (release waits for the stream,
    // which the box shares with its groups, so launches already enqueued finish first)
    for (lbm_sc_group* g : h->groups) {
        g->boxes.erase(std::remove(g->boxes.begin(), g->boxes.end(), h), g->boxes.end());
        g->dirty = true;
    }
    release(h);
}

}  // extern "C"
