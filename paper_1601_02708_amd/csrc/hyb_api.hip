// Runtime behind the C ABI of include/hyb.h: validates and uploads the
// problem, carves the caller's workspace, keeps the Schwarz/commit state
// machine of Algorithm 1 (Sec. 6.2) and enqueues the kernels on the
// caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hyb.h"
#include "hyb_impl.h"

using namespace hyb;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Scratch of hyb_diagnostics_noalloc: the row partials of the diagnostics
// reduction for lattices of up to kNoAllocMaxRows rows.  Every device the
// library runs on holds its own copy for the life of the process.  Host
// code never passes `scratch` itself to a kernel (on the host it names a
// stand-in, not device memory); it passes the device address that
// hipGetSymbolAddress returned for the current device, kept per device.
constexpr int kNoAllocMaxRows = 16384;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) double scratch[kDiagValues * kNoAllocMaxRows];
namespace {
std::mutex scratch_mu;
double *scratch_ptr[kMaxDevices] = {};

// Resolve the scratch's device address on `dev` (the current device), once.
hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = static_cast<double *>(p);
    return hipSuccess;
}

// Row pitch and plane stride (elements).  Rows start on 256-byte
// boundaries; planes are skewed by 128 elements so the nine streams of a
// sweep do not hit the same HBM channel offsets in lockstep.
int choose_pitch(int N) { return (int)align_up((size_t)N, 64); }
long long choose_plane(int N, int pitch) { return (long long)align_up((size_t)N * pitch, 64) + 128; }

bool valid_precision(int p) { return p == HYB_FP64 || p == HYB_FP32 || p == HYB_FP16S; }
size_t storage_bytes(int p) { return p == HYB_FP64 ? 8 : p == HYB_FP32 ? 4 : 2; }

// IEEE 754 binary32 <-> binary16 on the host, round to nearest even
// (the rounding the device conversion uses).
uint16_t f32_to_f16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    const uint32_t sign = (u >> 16) & 0x8000u;
    const uint32_t mag = u & 0x7fffffffu;
    if (mag >= 0x7f800000u) return (uint16_t)(sign | 0x7c00u | (mag > 0x7f800000u ? 0x200u : 0u));
    if (mag >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);        // >= 65520 rounds to infinity
    if (mag < 0x38800000u) {                                          // below 2^-14: subnormal or zero
        float f;
        std::memcpy(&f, &mag, 4);
        return (uint16_t)(sign | (uint32_t)std::nearbyint(f * 16777216.0f));   // exact scaling by 2^24
    }
    const uint32_t m = mag & 0x7fffffu;
    uint32_t h = (((mag >> 23) - 112u) << 10) | (m >> 13);
    const uint32_t rem = m & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h += 1u;     // carry may reach the exponent
    return (uint16_t)(sign | h);
}
float f16_to_f32(uint16_t h) {
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    const uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    if (e == 0) {
        const float f = (float)m * 5.9604644775390625e-08f;          // m * 2^-24
        return sign ? -f : f;
    }
    const uint32_t bits = sign | (e == 31 ? 0x7f800000u | (m << 13) : ((e + 112u) << 23) | (m << 13));
    float f;
    std::memcpy(&f, &bits, 4);
    return f;
}

int coarse_grid(int n) { return (n + 255) / 256; }
int coarse_grid8(int n) { return (8 * n + 255) / 256; }

// node-major [n][W*W] -> offset-major [W*W][n]
std::vector<double> offset_major(const std::vector<double> &c, int n, int w2) {
    std::vector<double> t(c.size());
    for (int node = 0; node < n; ++node)
        for (int o = 0; o < w2; ++o) t[(size_t)o * n + node] = c[(size_t)node * w2 + o];
    return t;
}

struct Layout {
    int pitch = 0;
    long long plane = 0;
    size_t f_bytes = 0;
    size_t u_bytes = 0;     // one plane of the arithmetic type (recorded u of a fine step)
    size_t mask = 0, vx = 0, vy = 0, kfield = 0, bc_kind = 0, bc_a = 0, bc_b = 0, c2f_idx = 0, c2f_w = 0;
    size_t fc_idx = 0, fc_w = 0, ufc = 0, A9 = 0, B9 = 0, AP = 0, P = 0, dkind = 0, vec = 0, partials = 0;
    size_t counters = 0, barrier = 0, kres = 0, diag = 0, total = 0;
    size_t APT = 0, PT = 0, c2fT_ptr = 0, c2fT_slot = 0, c2fT_w = 0, f2cT_node = 0, f2cT_ptr = 0, f2cT_c = 0;
    size_t f2cT_w = 0, fc_row = 0;
    // dissolving solids (hyb_lattice.dissolution): per-node mass, link flux
    // and solid flag; raw fine-to-coarse corners and fallbacks
    bool dissolve = false;
    size_t mass = 0, flux = 0, solid_now = 0, fcr_idx = 0, fcr_w = 0, fcr_fb = 0;
    // maximum-entropy closure at solid walls (hyb_lattice.wall_closure):
    // the wall normal's two FP32 planes
    bool wall = false;
    size_t wall_nx = 0, wall_ny = 0;
    size_t f2cD_node = 0, f2cD_ptr = 0, f2cD_c = 0, f2cD_m = 0;
    int n = 0, S = 0, grid = 0;
    size_t vec_len = 0;
};

Layout make_layout(const hyb_mesh *mesh, const hyb_lattice *lat, bool has_kfield) {
    Layout L;
    const int N = lat->N;
    const size_t elem = storage_bytes(lat->precision);
    L.pitch = choose_pitch(N);
    L.plane = choose_plane(N, L.pitch);
    L.f_bytes = align_up((size_t)9 * L.plane * elem, kAlign);
    L.u_bytes = align_up((size_t)L.plane * (lat->precision == HYB_FP64 ? 8 : 4), kAlign);
    const size_t nodes = (size_t)N * L.pitch;
    const size_t nslots = 4 * (size_t)(N - 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    L.mask = take(nodes * 2);
    L.vx = take(nodes * 4);
    L.vy = take(nodes * 4);
    L.kfield = has_kfield ? take(nodes * (lat->precision == HYB_FP64 ? 8 : 4)) : 0;
    L.bc_kind = take(nslots);
    L.bc_a = take(nslots * 8);
    L.bc_b = take(nslots * 8);
    L.counters = take(kCntSlots * 8);
    L.kres = take(sizeof(KrylovResult));
    L.diag = take(((size_t)kDiagValues * N + kDiagValues) * 8);   // row partials, then the result
    if (lat->wall_closure) {
        L.wall = true;
        L.wall_nx = take(nodes * 4);
        L.wall_ny = take(nodes * 4);
    }
    if (lat->dissolution) {
        L.dissolve = true;
        L.mass = take(nodes * 8);
        L.flux = take(nodes * 8);
        L.solid_now = take(nodes);
    }
    if (mesh) {
        const int M = mesh->M;
        L.n = (M + 1) * (M + 1);
        L.S = M + 1 + 2 * kCoarseHalo;
        L.grid = coarse_grid(L.n);
        L.vec_len = (size_t)L.S * L.S;
        L.c2f_idx = take(nslots * 4 * 4);
        L.c2f_w = take(nslots * 4 * 8);
        L.fc_idx = take((size_t)L.n * 4 * 4);
        L.fc_w = take((size_t)L.n * 4 * 8);
        L.ufc = take((size_t)L.n * 8);
        L.A9 = take((size_t)L.n * 9 * 8);
        L.B9 = take((size_t)L.n * 9 * 8);
        L.AP = take((size_t)L.n * kApW * kApW * 8);
        L.P = take((size_t)L.n * kSpaiW * kSpaiW * 8);
        L.dkind = take((size_t)L.n * 4);
        L.vec = take(12 * align_up(L.vec_len * 8, kAlign));
        L.partials = take((size_t)4 * kPartialValues * coarse_grid8(L.n) * 8);
        L.barrier = take(sizeof(KrylovState));
        // reverse mode: transposed stencils and transfer lists (at most 4
        // lattice nodes per Gamma_{f->c} node, at most n such nodes)
        L.APT = take((size_t)L.n * kApW * kApW * 8);
        L.PT = take((size_t)L.n * kSpaiW * kSpaiW * 8);
        L.c2fT_ptr = take(((size_t)L.n + 1) * 4);
        L.c2fT_slot = take(nslots * 4 * 4);
        L.c2fT_w = take(nslots * 4 * 8);
        L.f2cT_node = take((size_t)L.n * 4 * 4);
        L.f2cT_ptr = take(((size_t)L.n * 4 + 1) * 4);
        L.f2cT_c = take((size_t)L.n * 4 * 4);
        L.f2cT_w = take((size_t)L.n * 4 * 8);
        L.fc_row = take((size_t)L.n * 4);
        if (L.dissolve) {
            L.fcr_idx = take((size_t)L.n * 4 * 4);
            L.fcr_w = take((size_t)L.n * 4 * 8);
            L.fcr_fb = take((size_t)L.n * 4);
            // transposed superset: at most 5 entries per Gamma_{f->c} node
            L.f2cD_node = take((size_t)L.n * 5 * 4);
            L.f2cD_ptr = take(((size_t)L.n * 5 + 1) * 4);
            L.f2cD_c = take((size_t)L.n * 5 * 4);
            L.f2cD_m = take((size_t)L.n * 5 * 4);
        }
    }
    L.total = off;
    return L;
}

}  // namespace

struct hyb_handle {
    std::string err;
    // problem
    int N = 0, M = 0, eta = 1, clamp = 0;
    int prec = HYB_FP64;                // population storage (HYB_FP64 / FP32 / FP16S)
    int dev = 0;                        // device current at hyb_create
    bool fp64 = true, has_mesh = false, has_kfield = false;   // fp64: arithmetic type
    float hs_scale = 1.f, hs_inv = 1.f, hs_cref = 0.f;        // FP16S encoding
    std::vector<uint8_t> solid_host;    // [N*N] solid flags (readout zeroes solid nodes)
    double tau = 0, omega = 0, D = 0, kuni = 0;
    double x0 = 0, y0 = 0;
    hipStream_t stream = nullptr;
    Layout lay;
    void *f[3] = {nullptr, nullptr, nullptr};
    char *ws = nullptr;
    // workspace views
    uint16_t *mask = nullptr;
    float *vx = nullptr, *vy = nullptr;
    void *kfield = nullptr;
    int8_t *bc_kind = nullptr;
    double *bc_a = nullptr, *bc_b = nullptr;
    bool kinds_set = false;
    bool any_neumann = false;
    // maximum-entropy zero-flux closure at solid walls (hyb_set_wall_normals)
    bool wall_ws = false, wall_on = false;
    float *wall_nx = nullptr, *wall_ny = nullptr;
    int steps_per_launch = 4;          // most fine steps per sweep launch (fuse_steps)
    const void *rec_tape = nullptr;     // last forward recording (hyb_lbm_substeps_record)
    int rec_n = 0;
    // bumped by every call that changes the fine state, the interface
    // values or the rate field; the fine-step adjoint reads the recorded
    // start and end states from the handle's buffers, so it requires the
    // count the record left (rec_gen)
    unsigned long long gen = 0, rec_gen = 0;
    int *c2f_idx = nullptr, *fc_idx = nullptr;
    double *c2f_w = nullptr, *fc_w = nullptr, *ufc = nullptr;
    int nfc = 0;
    // reverse mode of the coarse half (hyb_step_record / hyb_step_adjoint)
    const double *apt = nullptr, *pt = nullptr;
    int *c2fT_ptr = nullptr, *c2fT_slot = nullptr, *f2cT_node = nullptr, *f2cT_ptr = nullptr, *f2cT_c = nullptr;
    int *fc_row = nullptr;
    double *c2fT_w = nullptr, *f2cT_w = nullptr;
    int f2cT_n = 0;
    const void *rec_step_tape = nullptr;    // last hyb_step_record
    // the record's start and end states stay in these buffers (checked by gen)
    int rec_step_f0 = -1, rec_step_out = -1;
    unsigned long long rec_step_gen = 0;
    int rec_step_passes = 0;
    // dissolving solids: workspace reserved (dissolve_ws), reaction on
    // (dissolve_on, from hyb_set_dissolution); flux_valid: the fine steps
    // since the last commit summed the link fluxes of the current pass
    bool dissolve_ws = false, dissolve_on = false, flux_valid = false, solid_host_stale = false;
    double kappa_s = 0.0, c_sat = 0.0;
    double *mass = nullptr, *flux = nullptr;
    uint8_t *solid_now = nullptr;
    int *fcr_idx = nullptr, *fcr_fb = nullptr;
    double *fcr_w = nullptr;
    int *f2cD_node = nullptr, *f2cD_ptr = nullptr, *f2cD_c = nullptr, *f2cD_m = nullptr;
    int f2cD_n = 0;
    std::vector<uint8_t> solid_init;    // [N*N] the geometry at hyb_create
    CoarseDev cd{};
    unsigned long long *counters = nullptr;
    KrylovResult *kres = nullptr;
    double *diag = nullptr;             // [kDiagValues N] row partials, then [kDiagValues] result
    // state machine
    int frozen = 0, cur = 0, jsub = 0;
    bool solved_this_step = false;
    int last_krylov_iters = 8;          // sizes the launch budget of the next solve
    int solve_budget = 0, solve_cap = 0;
    long long coarse_steps = 0, fine_steps = 0;
    unsigned long long seen_nonfinite = 0;
    // kernel timing (measurement only)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;       // pairs: [2k] begin, [2k+1] end
    std::vector<int> ev_launches;          // sweep launches bracketed by pair k
    size_t ev_used = 0;                    // pairs recorded and not yet read
    double timed_ms = 0.0;
    long long timed_launches = 0;

    // overlap of the deep interior tiles of each Schwarz pass's first
    // `overlap` two-step launches with the pass's transfers and coarse solve:
    // a second stream of the handle's own, one event per deep launch
    int overlap = HYB_OVERLAP_AUTO;
    hipStream_t side = nullptr;
    hipEvent_t ev_main = nullptr, ev_f2c = nullptr;
    // the previous pass's fine-to-coarse transfer, recorded after it reads
    // the fine state: when a pass is one launch, the next pass's deep tiles
    // only wait for that read (see hyb_step)
    hipEvent_t ev_read = nullptr;
    std::vector<hipEvent_t> ev_deep;
    // pinned host copy of the counters and the last coarse solve's result,
    // which every commit reads back (a copy into pageable memory stalls the
    // host for tens of microseconds per step)
    struct ReadBack {
        unsigned long long cnt[kCntSlots];
        KrylovResult kr;
    };
    ReadBack *rb = nullptr;
    // depth tuning (HYB_OVERLAP_AUTO): step times per depth, best of two
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    int tune_idx = 0, tuned_depth = -1;
    std::vector<float> tune_ms;

    ~hyb_handle() {
        if (ev_main) (void)hipEventDestroy(ev_main);
        if (ev_f2c) (void)hipEventDestroy(ev_f2c);
        if (ev_read) (void)hipEventDestroy(ev_read);
        if (rb) (void)hipHostFree(rb);
        if (ev_t0) (void)hipEventDestroy(ev_t0);
        if (ev_t1) (void)hipEventDestroy(ev_t1);
        for (hipEvent_t e : ev_deep) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
    // fold recorded pairs into the running sums (stream must be idle)
    hipError_t drain_events() {
        for (size_t k = 0; k < ev_used; ++k) {
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, ev_pool[2 * k], ev_pool[2 * k + 1]);
            if (e != hipSuccess) return e;
            timed_ms += ms;
            timed_launches += ev_launches[k];
        }
        ev_used = 0;
        return hipSuccess;
    }

    int fail(int code, const std::string &msg) {
        err = msg;
        return code;
    }
    int hip_fail(hipError_t e, const char *what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return HYB_EHIP;
    }
    LbmArgs lbm_args(int src, int dst) const {
        LbmArgs a{};
        a.src = f[src];
        a.dst = dst >= 0 ? f[dst] : nullptr;
        a.mask = mask;
        a.vx = vx;
        a.vy = vy;
        a.kfield = has_kfield ? kfield : nullptr;
        a.k = kuni;
        a.omega = omega;
        a.N = N;
        a.pitch = lay.pitch;
        a.plane = lay.plane;
        a.bc_kind = kinds_set ? bc_kind : nullptr;
        a.bc_a = bc_a;
        a.bc_b = bc_b;
        a.lam = 0.0;
        a.clamp = clamp;
        a.counters = counters;
        a.hs_scale = hs_scale;
        a.hs_inv = hs_inv;
        for (int q = 0; q < kQ; ++q) a.hs_wc[kWClass[q]] = (float)kW[q] * hs_cref;
        a.kappa_s = dissolve_on ? kappa_s : 0.0;
        a.c_sat = c_sat;
        a.flux = nullptr;
        a.flux_first = 0;
        a.mid = nullptr;
        a.wall_nx = wall_on ? wall_nx : nullptr;
        a.wall_ny = wall_on ? wall_ny : nullptr;
        return a;
    }
    // buffer that is neither the committed state nor `a`
    int spare(int a) const {
        for (int b = 0; b < 3; ++b)
            if (b != frozen && b != a) return b;
        return -1;
    }
};

#define HIP_TRY(h, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return (h)->hip_fail(e_, #call); \
    } while (0)

extern "C" {

int hyb_query(const hyb_mesh *mesh, const hyb_lattice *lat, size_t *f_bytes, size_t *ws_bytes) {
    if (!lat || lat->N < 3 || !valid_precision(lat->precision)) return HYB_EINVAL;
    if (mesh && mesh->M < 2) return HYB_EINVAL;
    // per-node kfield space is reserved; callers that pass none waste N^2 elements
    Layout L = make_layout(mesh, lat, true);
    if (f_bytes) *f_bytes = L.f_bytes;
    if (ws_bytes) *ws_bytes = L.total;
    return HYB_OK;
}

int hyb_create(const hyb_mesh *mesh, const hyb_lattice *lat, double D, const hyb_velocity *u,
               const hyb_reaction *k, hyb_handle **out) {
    if (!out) return HYB_EINVAL;
    *out = nullptr;
    hyb_handle *h = new hyb_handle();
    auto bail = [&](int code, const std::string &msg) {
        std::fprintf(stderr, "hyb_create: %s\n", msg.c_str());
        delete h;
        return code;
    };
    if (!lat || !u || !u->fine || !lat->u0) return bail(HYB_EINVAL, "lattice, velocity and u0 are required");
    const int N = lat->N;
    if (N < 3) return bail(HYB_EINVAL, "N must be >= 3");
    if (!valid_precision(lat->precision)) return bail(HYB_EINVAL, "unknown precision");
    if (!(D > 0.0)) return bail(HYB_EINVAL, "D must be > 0");
    if (lat->eta < 1) return bail(HYB_EINVAL, "eta must be >= 1");
    const double tau = lat->tau > 0.0 ? lat->tau : 0.5 + 3.0 * D;
    if (!(tau > 0.5)) return bail(HYB_EINVAL, "tau must exceed 1/2");
    const double kuni = k ? k->k : 0.0;
    if (!(kuni >= 0.0 && kuni < 1.0)) return bail(HYB_EINVAL, "reaction rate must lie in [0, 1)");
    if (k && k->k_field)
        for (size_t n = 0; n < (size_t)N * N; ++n)
            if (!(k->k_field[n] >= 0.0 && k->k_field[n] < 1.0))
                return bail(HYB_EINVAL, "reaction rates must lie in [0, 1)");
    if (mesh) {
        if (mesh->M < 2 || !(mesh->L > 0.0) || !mesh->d0 || !u->coarse || mesh->overlap_elems < 1 ||
            (mesh->outer_natural & ~15))
            return bail(HYB_EINVAL, "invalid mesh");
        if (lat->x0 < 0 || lat->y0 < 0 || lat->x0 + (N - 1) > mesh->L || lat->y0 + (N - 1) > mesh->L)
            return bail(HYB_EINVAL, "lattice patch must lie inside the coarse domain");
    }
    h->N = N;
    h->prec = lat->precision;
    {
        hipError_t e = hipGetDevice(&h->dev);
        if (e == hipSuccess) e = scratch_setup(h->dev);
        if (e != hipSuccess) return bail(HYB_EHIP, std::string("device set-up: ") + hipGetErrorString(e));
    }
    // measured fastest per storage type at pore2048: FP32 5 (84 GLUPS with
    // pairs, 107 with fours, 112 with fives), FP64 4 (58 -> 69; five steps
    // leave one 83 KB workgroup per CU: 52), FP16 shifted storage 4 (its
    // launches keep FP32 intermediates on chip: 82.4, 83.7, 88.9, 87.2 GLUPS
    // at 2, 3, 4, 5)
    h->steps_per_launch = lat->precision == HYB_FP16S ? 4 : lat->precision == HYB_FP64 ? 4 : 5;
    h->fp64 = lat->precision == HYB_FP64;
    h->tau = tau;
    h->omega = 1.0 / tau;
    h->D = D;
    h->eta = lat->eta;
    h->clamp = lat->bc_clamp ? 1 : 0;
    h->kuni = kuni;
    h->has_kfield = k && k->k_field;
    h->has_mesh = mesh != nullptr;
    h->M = mesh ? mesh->M : 0;
    h->x0 = lat->x0;
    h->y0 = lat->y0;
    h->stream = static_cast<hipStream_t>(lat->stream);
    // the side stream runs interior sweep tiles while the coarse solve runs on
    // the caller's stream (default priority; measured: restricting it to 7/8
    // or 4/5 of the CUs with a CU mask made the step 28% slower)
    if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_main, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_f2c, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_read, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&h->ev_t0) != hipSuccess || hipEventCreate(&h->ev_t1) != hipSuccess)
        return bail(HYB_EHIP, "could not create the handle's side stream and events");
    if (hipHostMalloc(reinterpret_cast<void **>(&h->rb), sizeof(hyb_handle::ReadBack), hipHostMallocDefault) !=
        hipSuccess)
        return bail(HYB_EHIP, "could not allocate the handle's pinned read-back buffer");
    h->lay = make_layout(mesh, lat, true);
    const Layout &L = h->lay;
    if ((long long)9 * L.plane >= (1LL << 31)) return bail(HYB_EINVAL, "lattice too large for 32-bit indexing");
    for (int b = 0; b < 3; ++b) {
        if (!lat->f_buf[b] || reinterpret_cast<uintptr_t>(lat->f_buf[b]) % kAlign)
            return bail(HYB_EINVAL, "population buffers must be non-null and 256-byte aligned");
        h->f[b] = lat->f_buf[b];
    }
    if (!lat->workspace || reinterpret_cast<uintptr_t>(lat->workspace) % kAlign)
        return bail(HYB_EINVAL, "workspace must be non-null and 256-byte aligned");
    h->ws = static_cast<char *>(lat->workspace);
    const int P = L.pitch;
    const size_t nodes = (size_t)N * P;

    // ---- host staging of geometry, velocity, reaction --------------------
    std::vector<uint16_t> mask(nodes, 0);
    auto solid = [&](int i, int j) { return lat->solid && lat->solid[(size_t)j * N + i]; };
    h->solid_host.assign((size_t)N * N, 0);
    if (lat->solid)
        for (size_t n = 0; n < (size_t)N * N; ++n) h->solid_host[n] = lat->solid[n] ? 1 : 0;
    h->solid_init = h->solid_host;
    if (h->prec == HYB_FP16S) {
        // c_ref = mean of u0 over the fluid nodes; scale = 2^s, the largest
        // power of two with (4/9) U 2^s <= 2^14, U = max(1, max |u0 - c_ref|)
        double sum = 0.0, cnt = 0.0;
        for (size_t n = 0; n < (size_t)N * N; ++n)
            if (!h->solid_host[n]) { sum += lat->u0[n]; cnt += 1.0; }
        const double cref = cnt > 0.0 ? sum / cnt : 0.0;
        double U = 1.0;
        for (size_t n = 0; n < (size_t)N * N; ++n)
            if (!h->solid_host[n]) U = std::max(U, std::fabs(lat->u0[n] - cref));
        if (!std::isfinite(U)) return bail(HYB_EINVAL, "u0 must be finite");
        const int s2 = (int)std::floor(std::log2(16384.0 / (4.0 / 9.0 * U)));
        h->hs_cref = (float)cref;
        h->hs_scale = std::ldexp(1.0f, s2);
        h->hs_inv = std::ldexp(1.0f, -s2);
    }
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            uint16_t m = 0;
            if (solid(i, j)) {
                if (i == 0 || j == 0 || i == N - 1 || j == N - 1)
                    return bail(HYB_EINVAL, "solid nodes on the lattice perimeter are not supported");
                m = kMaskSolid;
                for (int q = 1; q < kQ; ++q)
                    if (!solid(i + kCx[q], j + kCy[q])) m |= (uint16_t)(1u << q);
            } else {
                for (int q = 1; q < kQ; ++q) {
                    const int si = i - kCx[q], sj = j - kCy[q];
                    if (si >= 0 && si < N && sj >= 0 && sj < N && solid(si, sj)) m |= (uint16_t)(1u << q);
                }
            }
            mask[(size_t)j * P + i] = m;
        }
    std::vector<float> vxh(nodes, 0.f), vyh(nodes, 0.f);
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            const bool s = solid(i, j);
            vxh[(size_t)j * P + i] = s ? 0.f : u->fine[(size_t)j * N + i];
            vyh[(size_t)j * P + i] = s ? 0.f : u->fine[(size_t)N * N + (size_t)j * N + i];
        }
    h->mask = reinterpret_cast<uint16_t *>(h->ws + L.mask);
    h->vx = reinterpret_cast<float *>(h->ws + L.vx);
    h->vy = reinterpret_cast<float *>(h->ws + L.vy);
    h->kfield = h->ws + L.kfield;
    h->bc_kind = reinterpret_cast<int8_t *>(h->ws + L.bc_kind);
    h->bc_a = reinterpret_cast<double *>(h->ws + L.bc_a);
    h->bc_b = reinterpret_cast<double *>(h->ws + L.bc_b);
    h->counters = reinterpret_cast<unsigned long long *>(h->ws + L.counters);
    h->kres = reinterpret_cast<KrylovResult *>(h->ws + L.kres);
    h->diag = reinterpret_cast<double *>(h->ws + L.diag);
    if (L.wall) {
        h->wall_ws = true;
        h->wall_nx = reinterpret_cast<float *>(h->ws + L.wall_nx);
        h->wall_ny = reinterpret_cast<float *>(h->ws + L.wall_ny);
    }
    if (L.dissolve) {
        h->dissolve_ws = true;
        h->mass = reinterpret_cast<double *>(h->ws + L.mass);
        h->flux = reinterpret_cast<double *>(h->ws + L.flux);
        h->solid_now = reinterpret_cast<uint8_t *>(h->ws + L.solid_now);
    }
    hipStream_t st = h->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
#define CREATE_TRY(call)                                                              \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) return bail(HYB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
    CREATE_TRY(hipMemsetAsync(h->ws, 0, L.total, st));
    for (int b = 0; b < 3; ++b) CREATE_TRY(hipMemsetAsync(h->f[b], 0, L.f_bytes, st));
    CREATE_TRY(up(h->mask, mask.data(), nodes * 2));
    CREATE_TRY(up(h->vx, vxh.data(), nodes * 4));
    CREATE_TRY(up(h->vy, vyh.data(), nodes * 4));
    std::vector<uint8_t> solid_pitched;
    if (h->dissolve_ws) {
        solid_pitched.assign(nodes, 0);
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) solid_pitched[(size_t)j * P + i] = h->solid_host[(size_t)j * N + i];
        CREATE_TRY(up(h->solid_now, solid_pitched.data(), nodes));
    }
    if (h->has_kfield) {
        if (h->fp64) {
            std::vector<double> kf(nodes, 0.0);
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) kf[(size_t)j * P + i] = k->k_field[(size_t)j * N + i];
            CREATE_TRY(up(h->kfield, kf.data(), nodes * 8));
            CREATE_TRY(hipStreamSynchronize(st));
        } else {
            std::vector<float> kf(nodes, 0.f);
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) kf[(size_t)j * P + i] = (float)k->k_field[(size_t)j * N + i];
            CREATE_TRY(up(h->kfield, kf.data(), nodes * 4));
        }
        CREATE_TRY(hipStreamSynchronize(st));
    }

    // ---- coarse operator and interface lists --------------------------------
    if (mesh) {
        CoarseHost ch;
        std::string msg = build_coarse(mesh->M, mesh->L, D, kuni, (double)lat->eta, mesh->supg, u->coarse,
                                       mesh->overlap_elems, N, lat->x0, lat->y0, lat->solid, P, ch,
                                       mesh->outer_natural);
        if (!msg.empty()) return bail(HYB_EINVAL, msg);
        h->nfc = (int)ch.fc_nodes.size();
        h->c2f_idx = reinterpret_cast<int *>(h->ws + L.c2f_idx);
        h->c2f_w = reinterpret_cast<double *>(h->ws + L.c2f_w);
        h->fc_idx = reinterpret_cast<int *>(h->ws + L.fc_idx);
        h->fc_w = reinterpret_cast<double *>(h->ws + L.fc_w);
        h->ufc = reinterpret_cast<double *>(h->ws + L.ufc);
        CREATE_TRY(up(h->c2f_idx, ch.c2f_idx.data(), ch.c2f_idx.size() * 4));
        CREATE_TRY(up(h->c2f_w, ch.c2f_w.data(), ch.c2f_w.size() * 8));
        if (h->nfc) {
            CREATE_TRY(up(h->fc_idx, ch.fc_idx.data(), ch.fc_idx.size() * 4));
            CREATE_TRY(up(h->fc_w, ch.fc_w.data(), ch.fc_w.size() * 8));
        }
        CoarseDev &c = h->cd;
        c.M = mesh->M;
        c.n = L.n;
        c.S = L.S;
        c.grid = L.grid;
        c.grid8 = coarse_grid8(L.n);
        c.pstride = c.grid8;
        c.A9 = reinterpret_cast<const double *>(h->ws + L.A9);
        c.B9 = reinterpret_cast<const double *>(h->ws + L.B9);
        c.AP = reinterpret_cast<const double *>(h->ws + L.AP);
        c.P = reinterpret_cast<const double *>(h->ws + L.P);
        c.dkind = reinterpret_cast<const int *>(h->ws + L.dkind);
        c.outer_value = mesh->outer_value;
        c.ufc = h->ufc;
        const size_t vstride = align_up(L.vec_len * 8, kAlign);
        double *vec[12];
        for (int v = 0; v < 12; ++v) vec[v] = reinterpret_cast<double *>(h->ws + L.vec + v * vstride);
        c.xn = vec[0];
        c.x1 = vec[1];
        c.r = vec[2];
        c.rh = vec[3];
        c.p = vec[4];
        c.v = vec[5];
        c.s = vec[6];
        c.t = vec[7];
        c.y = vec[8];
        c.w = vec[9];
        c.z = vec[10];
        c.xprev = vec[11];
        c.partials = reinterpret_cast<double *>(h->ws + L.partials);
        c.state = reinterpret_cast<KrylovState *>(h->ws + L.barrier);
        c.result = h->kres;
        const std::vector<double> A9t = offset_major(ch.A9, L.n, 9), B9t = offset_major(ch.B9, L.n, 9);
        const std::vector<double> Pt = offset_major(ch.P, L.n, kSpaiW * kSpaiW);
        CREATE_TRY(up((void *)c.A9, A9t.data(), A9t.size() * 8));
        CREATE_TRY(up((void *)c.B9, B9t.data(), B9t.size() * 8));
        CREATE_TRY(up((void *)c.AP, ch.AP.data(), ch.AP.size() * 8));
        CREATE_TRY(up((void *)c.P, Pt.data(), Pt.size() * 8));
        CREATE_TRY(up((void *)c.dkind, ch.dkind.data(), ch.dkind.size() * 4));
        const std::vector<double> PTt = offset_major(ch.PT, L.n, kSpaiW * kSpaiW);
        h->apt = reinterpret_cast<const double *>(h->ws + L.APT);
        h->pt = reinterpret_cast<const double *>(h->ws + L.PT);
        h->c2fT_ptr = reinterpret_cast<int *>(h->ws + L.c2fT_ptr);
        h->c2fT_slot = reinterpret_cast<int *>(h->ws + L.c2fT_slot);
        h->c2fT_w = reinterpret_cast<double *>(h->ws + L.c2fT_w);
        h->f2cT_node = reinterpret_cast<int *>(h->ws + L.f2cT_node);
        h->f2cT_ptr = reinterpret_cast<int *>(h->ws + L.f2cT_ptr);
        h->f2cT_c = reinterpret_cast<int *>(h->ws + L.f2cT_c);
        h->f2cT_w = reinterpret_cast<double *>(h->ws + L.f2cT_w);
        h->fc_row = reinterpret_cast<int *>(h->ws + L.fc_row);
        h->f2cT_n = (int)ch.f2cT_node.size();
        if (h->f2cT_n > 4 * L.n) return bail(HYB_EINVAL, "internal: transposed transfer list too long");
        CREATE_TRY(up((void *)h->apt, ch.APT.data(), ch.APT.size() * 8));
        CREATE_TRY(up((void *)h->pt, PTt.data(), PTt.size() * 8));
        CREATE_TRY(up(h->c2fT_ptr, ch.c2fT_ptr.data(), ch.c2fT_ptr.size() * 4));
        CREATE_TRY(up(h->c2fT_slot, ch.c2fT_slot.data(), ch.c2fT_slot.size() * 4));
        CREATE_TRY(up(h->c2fT_w, ch.c2fT_w.data(), ch.c2fT_w.size() * 8));
        CREATE_TRY(up(h->f2cT_ptr, ch.f2cT_ptr.data(), ch.f2cT_ptr.size() * 4));
        if (h->f2cT_n) {
            CREATE_TRY(up(h->f2cT_node, ch.f2cT_node.data(), ch.f2cT_node.size() * 4));
            CREATE_TRY(up(h->f2cT_c, ch.f2cT_c.data(), ch.f2cT_c.size() * 4));
            CREATE_TRY(up(h->f2cT_w, ch.f2cT_w.data(), ch.f2cT_w.size() * 8));
        }
        if (h->nfc) CREATE_TRY(up(h->fc_row, ch.fc_nodes.data(), ch.fc_nodes.size() * 4));
        if (h->dissolve_ws) {
            h->fcr_idx = reinterpret_cast<int *>(h->ws + L.fcr_idx);
            h->fcr_w = reinterpret_cast<double *>(h->ws + L.fcr_w);
            h->fcr_fb = reinterpret_cast<int *>(h->ws + L.fcr_fb);
            h->f2cD_node = reinterpret_cast<int *>(h->ws + L.f2cD_node);
            h->f2cD_ptr = reinterpret_cast<int *>(h->ws + L.f2cD_ptr);
            h->f2cD_c = reinterpret_cast<int *>(h->ws + L.f2cD_c);
            h->f2cD_m = reinterpret_cast<int *>(h->ws + L.f2cD_m);
            h->f2cD_n = (int)ch.f2cD_node.size();
            if (ch.f2cD_c.size() > 5 * (size_t)L.n) return bail(HYB_EINVAL, "internal: transfer superset too long");
            if (h->nfc) {
                CREATE_TRY(up(h->fcr_idx, ch.fcr_idx.data(), ch.fcr_idx.size() * 4));
                CREATE_TRY(up(h->fcr_w, ch.fcr_w.data(), ch.fcr_w.size() * 8));
                CREATE_TRY(up(h->fcr_fb, ch.fcr_fb.data(), ch.fcr_fb.size() * 4));
                CREATE_TRY(up(h->f2cD_node, ch.f2cD_node.data(), ch.f2cD_node.size() * 4));
                CREATE_TRY(up(h->f2cD_ptr, ch.f2cD_ptr.data(), ch.f2cD_ptr.size() * 4));
                CREATE_TRY(up(h->f2cD_c, ch.f2cD_c.data(), ch.f2cD_c.size() * 4));
                CREATE_TRY(up(h->f2cD_m, ch.f2cD_m.data(), ch.f2cD_m.size() * 4));
            }
        }
        std::vector<double> xp(L.vec_len, 0.0);
        const int m1 = mesh->M + 1;
        for (int l = 0; l < m1; ++l)
            for (int kk = 0; kk < m1; ++kk) xp[(size_t)(l + kCoarseHalo) * L.S + kk + kCoarseHalo] = mesh->d0[l * m1 + kk];
        CREATE_TRY(up(c.xn, xp.data(), xp.size() * 8));
        CREATE_TRY(up(c.x1, xp.data(), xp.size() * 8));
        CREATE_TRY(up(c.xprev, xp.data(), xp.size() * 8));
        // host staging must stay alive until the copies ran
        CREATE_TRY(hipStreamSynchronize(st));
    }

    // ---- initial populations: f*(0) = collide(f^eq(u0)) ---------------------
    // u0 is staged in buffer 2, which is free until the first fine step
    CREATE_TRY(up(h->f[2], lat->u0, (size_t)N * N * 8));
    {
        LbmArgs a = h->lbm_args(2, 0);
        CREATE_TRY(launch_lbm_init(a, static_cast<const double *>(h->f[2]), h->prec, st));
    }
    CREATE_TRY(hipMemsetAsync(h->f[2], 0, L.f_bytes, st));
    CREATE_TRY(hipStreamSynchronize(st));
#undef CREATE_TRY
    h->frozen = 0;
    h->cur = 0;
    h->jsub = 0;
    *out = h;
    return HYB_OK;
}

int hyb_interface_exchange(hyb_handle *h, int direction) {
    if (!h) return HYB_EINVAL;
    ++h->gen;
    if (!h->has_mesh) return h->fail(HYB_EINVAL, "interface exchange needs a coarse mesh");
    if (direction == HYB_F2C) {
        LbmArgs a = h->lbm_args(h->cur, -1);
        if (h->dissolve_ws)
            HIP_TRY(h, launch_f2c_dynamic(a, h->fcr_idx, h->fcr_w, h->fcr_fb, h->nfc, h->ufc, h->prec, h->stream));
        else
            HIP_TRY(h, launch_f2c(a, h->fc_idx, h->fc_w, h->nfc, h->ufc, h->prec, h->stream));
    } else if (direction == HYB_C2F) {
        const double *xb = h->solved_this_step ? h->cd.x1 : h->cd.xn;
        HIP_TRY(h, launch_c2f(h->c2f_idx, h->c2f_w, 4 * (h->N - 1), h->cd.xn, xb, h->bc_a, h->bc_b, h->stream));
    } else {
        return h->fail(HYB_EINVAL, "unknown exchange direction");
    }
    return HYB_OK;
}

int hyb_coarse_step(hyb_handle *h, int max_iter) {
    if (!h) return HYB_EINVAL;
    if (!h->has_mesh) return h->fail(HYB_EINVAL, "coarse step needs a coarse mesh");
    if (max_iter <= 0) max_iter = 200;
    // first solve of a coarse step starts from the extrapolation
    // 2 d(t_n) - d(t_{n-1}) (d(t_n) itself at the first step); later Schwarz
    // passes start from the previous pass's solution
    if (!h->solved_this_step) HIP_TRY(h, launch_coarse_extrapolate(h->cd, h->stream));
    const double *guess = h->cd.x1;
    // iterations enqueued: a few more than the last solve needed (launches
    // after convergence are no-ops); hyb_commit reports a solve that ran out
    // of this budget and hyb_step then repeats the step with max_iter
    const int budget = std::min(max_iter, std::max(4, h->last_krylov_iters + 2));
    HIP_TRY(h, launch_coarse_rhs(h->cd, guess, h->stream));
    HIP_TRY(h, launch_coarse_solve(h->cd, guess, budget, max_iter, 1e-14, h->stream));
    h->solved_this_step = true;
    h->solve_budget = budget;
    h->solve_cap = max_iter;
    return HYB_OK;
}

}  // extern "C"

namespace {

// the two-step kernel addresses a population buffer with 32-bit byte
// offsets, so it serves buffers below 4 GiB (N up to about 11500 in FP64)
bool use_two_step(const hyb_handle *h) {
    const bool small_buf = 9.0 * (double)h->lay.plane * (double)storage_bytes(h->prec) < 4294967295.0;
    return !h->any_neumann && !h->wall_on && h->steps_per_launch >= 2 && small_buf;
}

// Most fine steps one launch of the forward sub-stepping takes: the
// handle's steps per launch where multi-step launches apply, else 1.
int fuse_steps(const hyb_handle *h) {
    if (!use_two_step(h)) return 1;
    return h->steps_per_launch;
}

// Fine steps of the next launch when `rem` steps of the call remain, never
// leaving a lone single step where it can be avoided: with three-step
// launches a remainder of 4 is taken as 2 + 2 (eta = 10: 3, 3, 2, 2); with
// four-step launches remainders of 5 and 6 start with a 3 (eta = 10: 4, 3, 3).
int plan_take(int fuse, int rem) {
    if (rem <= 1 || fuse == 1) return rem < 1 ? 0 : 1;
    if (fuse == 2 || rem == 2) return 2;
    if (fuse == 3) return rem == 4 ? 2 : 3;
    if (fuse == 4) return rem == 3 || rem == 5 || rem == 6 ? 3 : 4;
    // five: a remainder of 6 as 3 + 3, 7 as 4 + 3, 8 as 4 + 4, 9 as 5 + 4
    return rem == 6 ? 3 : rem == 7 || rem == 8 ? 4 : rem >= 5 ? 5 : rem;
}

// Ring of the overlap rectangles of a pass: a K-step kernel reads K-1 nodes
// beyond its tile, and every launch of a pass uses the widest ring so that
// the rectangles of successive launches nest.
int pass_ring(const hyb_handle *h) { return fuse_steps(h) >= 3 ? fuse_steps(h) - 1 : 1; }

// largest overlap depth hyb_step may use: the leading multi-step launches of
// a pass (none with dissolving solids, whose sweeps run whole-patch launches)
int overlap_dmax(const hyb_handle *h) {
    if (!use_two_step(h) || h->dissolve_on) return 0;
    const int fuse = fuse_steps(h);
    int k = 0;
    for (int rem = h->eta; rem > 0; ++k) {
        const int t = plan_take(fuse, rem);
        if (t < 2) break;
        rem -= t;
    }
    return k;
}

// One multi-step launch of `take` fine steps (2, 3 or 4) from a.src to a.dst,
// fine steps j0 + 1 .. j0 + take of the pass (interface weights (j0+1)/eta,
// ...).
hipError_t launch_fused(const hyb_handle *h, LbmArgs a, int j0, int take, hipStream_t s, int part, int depth) {
    a.lam = (double)(j0 + 1) / (double)h->eta;
    a.lam2 = (double)(j0 + 2) / (double)h->eta;
    a.lam3 = (double)(j0 + 3) / (double)h->eta;
    a.lam4 = (double)(j0 + 4) / (double)h->eta;
    a.lam5 = (double)(j0 + 5) / (double)h->eta;
    if (take >= 3) return launch_lbm_stepk(a, h->prec, take, s, part, depth, pass_ring(h));
    return launch_lbm_step2(a, h->prec, s, part, depth, pass_ring(h));
}

// the host copy of the solid flags after commits that may have converted
// solids (waits for the stream)
hipError_t refresh_solid_host(hyb_handle *h) {
    if (!h->solid_host_stale) return hipSuccess;
    const int N = h->N, P = h->lay.pitch;
    std::vector<uint8_t> pitched((size_t)N * P);
    hipError_t e = hipMemcpyAsync(pitched.data(), h->solid_now, pitched.size(), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) h->solid_host[(size_t)j * N + i] = pitched[(size_t)j * P + i];
    h->solid_host_stale = false;
    return hipSuccess;
}

// n_sub fine steps.  first_dst >= 0 (with restart): destination of the first
// launch; deep = K > 0: the first K launches are two-step launches whose
// deep tiles (part 1 of depth j for launch j = 0..K-1) were already enqueued
// on the side stream (prelaunch_deep), so only their other tiles (part 2 of
// the same depth) are launched here: launch j after the side stream's event
// for launch j-1 (its halo reaches into the deep tiles of launch j-1), and
// the first launch after them (or, when there is none, the end of the
// call) after the event for launch K-1.
int substeps_impl(hyb_handle *h, int n_sub, int restart, int first_dst, int deep) {
    if (n_sub < 0) return h->fail(HYB_EINVAL, "n_sub must be >= 0");
    if (restart) {
        h->cur = h->frozen;
        h->jsub = 0;
    }
    if (h->jsub + n_sub > h->eta) return h->fail(HYB_EINVAL, "fine steps would pass the end of the coarse step");
    // kernel timing: when every perimeter slot is Dirichlet only sweep
    // kernels are launched, back to back, so one event pair brackets the
    // batch (after split launches, which overlap other work); the general
    // path brackets each interior kernel alone (its perimeter kernel follows
    // it)
    const bool timed = h->timing && h->N > 2 && n_sub > 0;
    const bool general = h->any_neumann || h->wall_on;
    const int fuse = fuse_steps(h);
    auto take_pair = [&](hipEvent_t *e0, hipEvent_t *e1) -> hipError_t {
        if (2 * (h->ev_used + 1) > h->ev_pool.size()) {
            for (int k = 0; k < 2; ++k) {
                hipEvent_t e;
                hipError_t err = hipEventCreate(&e);
                if (err != hipSuccess) return err;
                h->ev_pool.push_back(e);
            }
            h->ev_launches.push_back(0);
        }
        *e0 = h->ev_pool[2 * h->ev_used];
        *e1 = h->ev_pool[2 * h->ev_used + 1];
        h->ev_launches[h->ev_used] = 0;
        h->ev_used += 1;
        return hipSuccess;
    };
    hipEvent_t g0 = nullptr, g1 = nullptr;
    size_t gslot = 0;
    int launch = 0;
    for (int s = 0; s < n_sub; ++launch) {
        const bool first = s == 0;
        const int dst = (first && first_dst >= 0) ? first_dst
                        : h->cur == h->frozen ? h->spare(-1) : h->spare(h->cur);
        LbmArgs a = h->lbm_args(h->cur, dst);
        a.lam = (double)(h->jsub + 1) / (double)h->eta;
        if (h->dissolve_on) {
            // the pass's first step starts the sums of its link fluxes
            a.flux = h->flux;
            a.flux_first = h->jsub == 0;
            h->flux_valid = true;
        }
        const int take = plan_take(fuse, n_sub - s);
        const bool split_now = launch < deep;
        if (split_now && take < 2) return h->fail(HYB_EINVAL, "internal: split launch is not a multi-step launch");
        // the side stream's deep tiles this launch depends on
        if (deep > 0 && launch >= 1 && launch <= deep)
            HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_deep[launch - 1], 0));
        if (timed && !general && !g0 && !split_now) {
            HIP_TRY(h, take_pair(&g0, &g1));
            gslot = h->ev_used - 1;
            HIP_TRY(h, hipEventRecord(g0, h->stream));
        }
        if (take >= 2) {
            HIP_TRY(h, launch_fused(h, a, h->jsub, take, h->stream, split_now ? 2 : 0, split_now ? launch : 0));
        } else {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed && general) {
                HIP_TRY(h, take_pair(&e0, &e1));
                h->ev_launches[h->ev_used - 1] = 1;
            }
            HIP_TRY(h, launch_lbm_step(a, h->prec, general, h->stream, e0, e1));
        }
        if (g0 && !split_now) h->ev_launches[gslot] += 1;
        h->cur = dst;
        h->jsub += take;
        h->fine_steps += take;
        s += take;
    }
    if (g1) HIP_TRY(h, hipEventRecord(g1, h->stream));
    // when every launch was split, no later launch joined the side stream:
    // join it here, so the pass ends with its last buffer complete
    if (deep > 0 && launch <= deep) HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_deep[deep - 1], 0));
    return HYB_OK;
}

// Enqueue, on the side stream, the deep tiles of the first `deep` two-step
// launches of a Schwarz pass: launch j (fine steps 2j+1, 2j+2) covers the
// interior rectangle of depth j, from the frozen state into dst for j = 0
// and then alternating between dst and the other free buffer.  They read
// only earlier deep tiles, the lattice fields and no interface value, so
// they run while the pass's coarse solve is in flight.  Launch 0 follows
// everything enqueued on the caller's stream before the call; the later
// launches also follow the fine-to-coarse transfer, which the caller
// enqueues between the two calls (the buffer it reads may be the one that
// launch 1 writes).
int prelaunch_deep(hyb_handle *h, int dst, int deep, bool after_f2c, bool after_read = false) {
    // the pass's launch plan (as substeps_impl takes it for eta steps):
    // launch j covers fine steps start[j] + 1 .. start[j] + take[j]
    const int fuse = fuse_steps(h);
    std::vector<int> start, take;
    for (int rem = h->eta, j0 = 0; rem > 0 && (int)take.size() < deep;) {
        const int t = plan_take(fuse, rem);
        if (t < 2) return h->fail(HYB_EINVAL, "internal: overlap depth beyond the pass's multi-step launches");
        start.push_back(j0);
        take.push_back(t);
        j0 += t;
        rem -= t;
    }
    if ((int)take.size() < deep) return h->fail(HYB_EINVAL, "internal: overlap depth beyond the pass's launches");
    auto launch = [&](int j, int src_buf, int dst_buf) {
        return launch_fused(h, h->lbm_args(src_buf, dst_buf), start[j], take[j], h->side, 1, j);
    };
    while ((int)h->ev_deep.size() < deep) {
        hipEvent_t e;
        HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->ev_deep.push_back(e);
    }
    if (!after_f2c) {
        // after_read: the pass's first launch is its only one, so its deep
        // tiles overwrite only the buffer the previous pass's fine-to-coarse
        // transfer read (they read the frozen state, and the previous pass
        // wrote the other buffer): waiting for that read suffices
        if (after_read) {
            HIP_TRY(h, hipStreamWaitEvent(h->side, h->ev_read, 0));
        } else {
            HIP_TRY(h, hipEventRecord(h->ev_main, h->stream));
            HIP_TRY(h, hipStreamWaitEvent(h->side, h->ev_main, 0));
        }
        HIP_TRY(h, launch(0, h->frozen, dst));
        HIP_TRY(h, hipEventRecord(h->ev_deep[0], h->side));
        return HYB_OK;
    }
    if (deep < 2) return HYB_OK;
    HIP_TRY(h, hipEventRecord(h->ev_f2c, h->stream));
    HIP_TRY(h, hipStreamWaitEvent(h->side, h->ev_f2c, 0));
    int src = dst;
    for (int j = 1; j < deep; ++j) {
        const int out = h->spare(src);
        HIP_TRY(h, launch(j, src, out));
        HIP_TRY(h, hipEventRecord(h->ev_deep[j], h->side));
        src = out;
    }
    return HYB_OK;
}

}  // namespace

extern "C" {

int hyb_lbm_substeps(hyb_handle *h, int n_sub, int restart) {
    if (!h) return HYB_EINVAL;
    ++h->gen;
    return substeps_impl(h, n_sub, restart, -1, 0);
}

int hyb_set_overlap(hyb_handle *h, int depth) {
    if (!h) return HYB_EINVAL;
    if (depth < HYB_OVERLAP_AUTO) return h->fail(HYB_EINVAL, "overlap depth must be >= 0 or HYB_OVERLAP_AUTO");
    h->overlap = depth;
    h->tune_idx = 0;
    h->tuned_depth = -1;
    h->tune_ms.clear();
    return HYB_OK;
}

int hyb_commit(hyb_handle *h) {
    if (!h) return HYB_EINVAL;
    ++h->gen;
    HIP_TRY(h, hipMemcpyAsync(h->rb->cnt, h->counters, sizeof(h->rb->cnt), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(&h->rb->kr, h->kres, sizeof(KrylovResult), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, h->drain_events());
    unsigned long long cnt[kCntSlots];
    for (int k = 0; k < kCntSlots; ++k) cnt[k] = h->rb->cnt[k];
    const KrylovResult kr = h->rb->kr;
    if (cnt[kCntNonfinite] != h->seen_nonfinite) {
        h->seen_nonfinite = cnt[kCntNonfinite];
        return h->fail(HYB_ENONFINITE, "non-finite concentration in the fine subdomain; state not committed");
    }
    if (h->solved_this_step) h->last_krylov_iters = kr.iters;
    if (h->solved_this_step && !kr.converged) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "coarse solve did not converge (%d iterations, relres %.3e)", kr.iters,
                      kr.relres);
        return h->fail(HYB_ENOCONV, buf);
    }
    h->frozen = h->cur;
    h->jsub = 0;
    if (h->dissolve_on && h->flux_valid) {
        // the last pass's link fluxes debit the solids; exhausted ones turn fluid
        LbmArgs a = h->lbm_args(h->frozen, h->frozen);
        a.flux = h->flux;
        HIP_TRY(h, launch_dissolve_commit(a, h->prec, h->mass, h->solid_now, h->mask, h->stream));
        h->solid_host_stale = true;
    }
    h->flux_valid = false;
    if (h->solved_this_step) {
        // d(t_{n-1}) <- d(t_n) <- new solution; the old d(t_{n-1}) buffer is free
        double *old_prev = h->cd.xprev;
        h->cd.xprev = h->cd.xn;
        h->cd.xn = h->cd.x1;
        h->cd.x1 = old_prev;
    }
    h->solved_this_step = false;
    h->coarse_steps += 1;
    return HYB_OK;
}

int hyb_step(hyb_handle *h, int max_schwarz) {
    if (!h) return HYB_EINVAL;
    ++h->gen;
    if (!h->has_mesh) return h->fail(HYB_EINVAL, "hyb_step needs a coarse mesh");
    if (max_schwarz < 1) return h->fail(HYB_EINVAL, "max_schwarz must be >= 1");
    // overlap depth: fixed, tuned, or the next candidate while tuning (one
    // untimed step, then three rounds over depths 0 .. D, each step timed on
    // the caller's stream; the fastest of each depth's three counts)
    const int dmax = overlap_dmax(h);
    const int ncand = dmax + 1;
    int depth = std::min(h->overlap, dmax);
    const bool tuning = h->overlap == HYB_OVERLAP_AUTO && dmax > 0 && h->tuned_depth < 0;
    if (h->overlap == HYB_OVERLAP_AUTO)
        depth = dmax == 0 ? 0 : !tuning ? h->tuned_depth : h->tune_idx == 0 ? 0 : (h->tune_idx - 1) % ncand;
    if (tuning) HIP_TRY(h, hipEventRecord(h->ev_t0, h->stream));
    int rc = HYB_OK;
    // a pass of one multi-step launch (eta fine steps in one launch)
    const bool one_launch = fuse_steps(h) >= 2 && plan_take(fuse_steps(h), h->eta) == h->eta;
    for (int attempt = 0; attempt < 2; ++attempt) {
        h->cur = h->frozen;
        h->jsub = 0;
        h->solved_this_step = false;
        const int deep = depth;
        for (int it = 0; it < max_schwarz; ++it) {
            // the pass's first launch writes a buffer that is neither the
            // frozen state nor the one the fine-to-coarse transfer reads
            int first_dst = -1;
            if (deep > 0) {
                first_dst = h->cur == h->frozen ? h->spare(-1) : h->spare(h->cur);
                if ((rc = prelaunch_deep(h, first_dst, deep, false, it > 0 && one_launch)) != HYB_OK) return rc;
            }
            if ((rc = hyb_interface_exchange(h, HYB_F2C)) != HYB_OK) return rc;
            if (one_launch && deep > 0) HIP_TRY(h, hipEventRecord(h->ev_read, h->stream));
            if (deep > 1 && (rc = prelaunch_deep(h, first_dst, deep, true)) != HYB_OK) return rc;
            if ((rc = hyb_coarse_step(h, 200)) != HYB_OK) return rc;
            if ((rc = hyb_interface_exchange(h, HYB_C2F)) != HYB_OK) return rc;
            if ((rc = substeps_impl(h, h->eta, 1, first_dst, deep)) != HYB_OK) return rc;
        }
        if (tuning) HIP_TRY(h, hipEventRecord(h->ev_t1, h->stream));
        rc = hyb_commit(h);
        // a coarse solve that ran out of its launch budget (not of max_iter)
        // is repeated once from the untouched committed state
        if (rc != HYB_ENOCONV || h->solve_budget >= h->solve_cap) break;
        h->last_krylov_iters = h->solve_cap;
    }
    if (tuning && rc == HYB_OK) {
        // the commit synchronised the stream, so both events are complete;
        // a repeated step is timed whole and counts like any other
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));
        if ((int)h->tune_ms.size() != ncand) h->tune_ms.assign(ncand, 1e30f);
        if (h->tune_idx > 0) h->tune_ms[depth] = std::min(h->tune_ms[depth], ms);
        if (++h->tune_idx == 1 + 3 * ncand)
            h->tuned_depth = (int)(std::min_element(h->tune_ms.begin(), h->tune_ms.end()) - h->tune_ms.begin());
    }
    return rc;
}

int hyb_set_boundary(hyb_handle *h, const int8_t *kind, const double *a, const double *b) {
    if (!h || !a) return HYB_EINVAL;
    ++h->gen;
    const size_t ns = 4 * (size_t)(h->N - 1);
    if (kind) {
        for (size_t p = 0; p < ns; ++p)
            if (kind[p] != HYB_BC_DIRICHLET && kind[p] != HYB_BC_NEUMANN)
                return h->fail(HYB_EINVAL, "unknown boundary kind");
        HIP_TRY(h, hipMemcpyAsync(h->bc_kind, kind, ns, hipMemcpyHostToDevice, h->stream));
        h->kinds_set = true;
        h->any_neumann = false;
        for (size_t p = 0; p < ns; ++p) h->any_neumann |= kind[p] == HYB_BC_NEUMANN;
    } else {
        h->kinds_set = false;
        h->any_neumann = false;
    }
    HIP_TRY(h, hipMemcpyAsync(h->bc_a, a, ns * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->bc_b, b ? b : a, ns * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return HYB_OK;
}

int hyb_concentration(hyb_handle *h, int which, double *out, int out_is_device) {
    if (!h || !out) return HYB_EINVAL;
    if (which == HYB_FINE) {
        const size_t bytes = (size_t)h->N * h->N * 8;
        double *dev = out_is_device ? out : static_cast<double *>(h->f[h->spare(h->cur == h->frozen ? -1 : h->cur)]);
        LbmArgs a = h->lbm_args(h->cur, -1);
        HIP_TRY(h, launch_concentration(a, dev, h->prec, h->stream));
        if (!out_is_device) HIP_TRY(h, hipMemcpyAsync(out, dev, bytes, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return HYB_OK;
    }
    if (which == HYB_COARSE) {
        if (!h->has_mesh) return h->fail(HYB_EINVAL, "no coarse mesh");
        const int m1 = h->M + 1;
        const double *src = h->solved_this_step ? h->cd.x1 : h->cd.xn;
        const size_t rowb = (size_t)m1 * 8;
        HIP_TRY(h, hipMemcpy2DAsync(out, rowb, src + (size_t)kCoarseHalo * h->cd.S + kCoarseHalo, (size_t)h->cd.S * 8,
                                    rowb, m1, out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                    h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        return HYB_OK;
    }
    return h->fail(HYB_EINVAL, "unknown field");
}

int hyb_populations_device(hyb_handle *h, double *out) {
    if (!h || !out) return HYB_EINVAL;
    if (h->prec == HYB_FP16S) return h->fail(HYB_EINVAL, "device readout supports HYB_FP64 and HYB_FP32 storage");
    LbmArgs a = h->lbm_args(h->cur, -1);
    HIP_TRY(h, launch_adjoint_pack(a, h->prec, out, h->f[h->cur], false, h->stream));
    return HYB_OK;
}

int hyb_get_populations(hyb_handle *h, double *out) {
    if (!h || !out) return HYB_EINVAL;
    if (refresh_solid_host(h) != hipSuccess) return h->fail(HYB_EHIP, "could not read the solid flags");
    const int N = h->N, P = h->lay.pitch;
    const size_t elem = storage_bytes(h->prec);
    std::vector<char> stage((size_t)9 * h->lay.plane * elem);
    HIP_TRY(h, hipMemcpyAsync(stage.data(), h->f[h->cur], stage.size(), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int q = 0; q < kQ; ++q) {
        const float wc = (float)kW[q] * h->hs_cref;
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const size_t s = (size_t)q * h->lay.plane + (size_t)j * P + i;
                double v;
                if (h->solid_host[(size_t)j * N + i]) v = 0.0;
                else if (h->prec == HYB_FP64) v = reinterpret_cast<const double *>(stage.data())[s];
                else if (h->prec == HYB_FP32) v = reinterpret_cast<const float *>(stage.data())[s];
                else v = f16_to_f32(reinterpret_cast<const uint16_t *>(stage.data())[s]) * h->hs_inv + wc;
                out[(size_t)q * N * N + (size_t)j * N + i] = v;
            }
    }
    return HYB_OK;
}

int hyb_set_populations(hyb_handle *h, const double *fin) {
    if (!h || !fin) return HYB_EINVAL;
    ++h->gen;
    const int N = h->N, P = h->lay.pitch;
    const size_t elem = storage_bytes(h->prec);
    std::vector<char> stage((size_t)9 * h->lay.plane * elem, 0);
    for (int q = 0; q < kQ; ++q) {
        const float wc = (float)kW[q] * h->hs_cref;
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const size_t s = (size_t)q * h->lay.plane + (size_t)j * P + i;
                const double v = fin[(size_t)q * N * N + (size_t)j * N + i];
                if (h->prec == HYB_FP64) reinterpret_cast<double *>(stage.data())[s] = v;
                else if (h->prec == HYB_FP32) reinterpret_cast<float *>(stage.data())[s] = (float)v;
                else reinterpret_cast<uint16_t *>(stage.data())[s] = f32_to_f16(((float)v - wc) * h->hs_scale);
            }
    }
    HIP_TRY(h, hipMemcpyAsync(h->f[h->frozen], stage.data(), stage.size(), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->cur = h->frozen;
    h->jsub = 0;
    return HYB_OK;
}

int hyb_set_coarse(hyb_handle *h, const double *d) {
    if (!h || !d) return HYB_EINVAL;
    if (!h->has_mesh) return h->fail(HYB_EINVAL, "no coarse mesh");
    const int m1 = h->M + 1;
    std::vector<double> xp(h->lay.vec_len, 0.0);
    for (int l = 0; l < m1; ++l)
        for (int kk = 0; kk < m1; ++kk) xp[(size_t)(l + kCoarseHalo) * h->cd.S + kk + kCoarseHalo] = d[l * m1 + kk];
    for (double *dst : {h->cd.xn, h->cd.x1, h->cd.xprev})
        HIP_TRY(h, hipMemcpyAsync(dst, xp.data(), xp.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->solved_this_step = false;
    h->cur = h->frozen;
    h->jsub = 0;
    return HYB_OK;
}

int hyb_set_reaction_field(hyb_handle *h, const double *k_field) {
    if (!h || !k_field) return HYB_EINVAL;
    ++h->gen;
    const int N = h->N;
    const size_t P = (size_t)h->lay.pitch, nodes = (size_t)N * P;
    for (size_t n = 0; n < (size_t)N * N; ++n)
        if (!(k_field[n] >= 0.0 && k_field[n] < 1.0)) return h->fail(HYB_EINVAL, "reaction rates must lie in [0, 1)");
    if (h->fp64) {
        std::vector<double> kf(nodes, 0.0);
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) kf[(size_t)j * P + i] = k_field[(size_t)j * N + i];
        HIP_TRY(h, hipMemcpyAsync(h->kfield, kf.data(), nodes * 8, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    } else {
        std::vector<float> kf(nodes, 0.f);
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) kf[(size_t)j * P + i] = (float)k_field[(size_t)j * N + i];
        HIP_TRY(h, hipMemcpyAsync(h->kfield, kf.data(), nodes * 4, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    h->has_kfield = true;
    return HYB_OK;
}

int hyb_set_outer_value(hyb_handle *h, double value) {
    if (!h) return HYB_EINVAL;
    if (!h->has_mesh) return h->fail(HYB_EINVAL, "no coarse mesh");
    if (!std::isfinite(value)) return h->fail(HYB_EINVAL, "outer value must be finite");
    h->cd.outer_value = value;
    return HYB_OK;
}

int hyb_diagnostics(hyb_handle *h, double *out, int out_is_device) {
    if (!h || !out) return HYB_EINVAL;
    LbmArgs a = h->lbm_args(h->cur, -1);
    double *res = out_is_device ? out : h->diag + (size_t)kDiagValues * h->N;
    HIP_TRY(h, launch_diagnostics(a, h->prec, h->diag, res, h->stream));
    if (!out_is_device) {
        HIP_TRY(h, hipMemcpyAsync(out, res, kDiagValues * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return HYB_OK;
}

int hyb_diagnostics_noalloc(hyb_handle *h, double *out) {
    if (!h || !out) return HYB_EINVAL;
    if (h->N > kNoAllocMaxRows)
        return h->fail(HYB_EINVAL, "hyb_diagnostics_noalloc: the lattice has more rows than its static scratch "
                                   "holds (N <= 16384)");
    double *part = h->dev >= 0 && h->dev < kMaxDevices ? scratch_ptr[h->dev] : nullptr;
    if (!part) return h->fail(HYB_EHIP, "hyb_diagnostics_noalloc: no scratch address for this device");
    LbmArgs a = h->lbm_args(h->cur, -1);
    HIP_TRY(h, launch_diagnostics(a, h->prec, part, out, h->stream));
    return HYB_OK;
}

int hyb_stats(hyb_handle *h, hyb_run_stats *out) {
    if (!h || !out) return HYB_EINVAL;
    unsigned long long cnt[kCntSlots];
    KrylovResult kr{};
    double dg[kDiagValues];
    const int rc = hyb_diagnostics(h, dg, 0);
    if (rc != HYB_OK) return rc;
    HIP_TRY(h, hipMemcpyAsync(cnt, h->counters, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(&kr, h->kres, sizeof(kr), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out->mass = dg[0];
    out->min_f = dg[1];
    out->h_function = dg[2];
    out->infeasible = (int64_t)cnt[kCntInfeasible];
    out->nonfinite = (int64_t)cnt[kCntNonfinite];
    out->krylov_iters = kr.iters;
    out->krylov_converged = kr.converged;
    out->krylov_relres = kr.relres;
    out->coarse_steps = h->coarse_steps;
    out->fine_steps = h->fine_steps;
    const int dmax = overlap_dmax(h);
    out->overlap_depth = h->overlap != HYB_OVERLAP_AUTO ? std::min(h->overlap, dmax)
                         : dmax == 0 ? 0 : h->tuned_depth;
    out->pad = 0;
    return HYB_OK;
}

int hyb_adjoint_query(const hyb_handle *h, int n_sub, size_t *tape_bytes) {
    if (!h || !tape_bytes || n_sub < 1) return HYB_EINVAL;
    // states f*(0) .. f*(n_sub), two adjoint fields and one scratch field,
    // then u of the collisions of fine steps 1 .. n_sub
    *tape_bytes = (size_t)(n_sub + 4) * h->lay.f_bytes + (size_t)n_sub * h->lay.u_bytes;
    return HYB_OK;
}

int hyb_lbm_substeps_record(hyb_handle *h, int n_sub, void *tape) {
    if (h && h->wall_on) return h->fail(HYB_EINVAL, "the adjoint supports bounce-back walls only");
    if (!h) return HYB_EINVAL;
    ++h->gen;
    if (h->prec == HYB_FP16S) return h->fail(HYB_EINVAL, "the adjoint supports HYB_FP64 and HYB_FP32 storage");
    if (h->any_neumann) return h->fail(HYB_EINVAL, "the adjoint supports Dirichlet perimeter slots only");
    if (n_sub < 1 || n_sub > h->eta) return h->fail(HYB_EINVAL, "n_sub must lie in 1..eta");
    if (!tape || reinterpret_cast<uintptr_t>(tape) % kAlign) return h->fail(HYB_EINVAL, "tape must be 256-byte aligned");
    const size_t fb = h->lay.f_bytes;
    // f*(0) is the committed buffer and f*(n_sub) goes straight to a spare
    // buffer of the handle, which becomes its current state; the states in
    // between go to the tape
    const int dst = h->spare(-1);
    auto state = [&](int t) -> void * {
        if (t == 0) return h->f[h->frozen];
        if (t == n_sub) return h->f[dst];
        return static_cast<char *>(tape) + (size_t)t * fb;
    };
    // u of step t's collision (t = 1 .. n_sub), after the states and the
    // three adjoint fields (not with dissolving solids, whose reversed steps
    // read the states)
    auto uplane = [&](int t) -> void * {
        if (h->dissolve_on) return nullptr;
        return static_cast<char *>(tape) + (size_t)(n_sub + 4) * fb + (size_t)(t - 1) * h->lay.u_bytes;
    };
    // pairs of fine steps in one launch that also stores the state between
    // them, while the two-step sweep serves (with dissolving solids the pair
    // also sums both steps' link fluxes)
    const bool pairs = use_two_step(h);
    for (int t = 0; t < n_sub;) {
        LbmArgs a = h->lbm_args(h->frozen, -1);
        a.src = state(t);
        a.lam = (double)(t + 1) / (double)h->eta;
        a.u_out = uplane(t + 1);
        if (h->dissolve_on) {
            a.flux = h->flux;
            a.flux_first = t == 0;
            h->flux_valid = true;
        }
        if (pairs && t + 2 <= n_sub) {
            a.mid = state(t + 1);
            a.dst = state(t + 2);
            a.u_out2 = uplane(t + 2);
            a.lam2 = (double)(t + 2) / (double)h->eta;
            HIP_TRY(h, launch_lbm_step2(a, h->prec, h->stream));
            t += 2;
            continue;
        }
        a.dst = state(t + 1);
        HIP_TRY(h, launch_lbm_step(a, h->prec, false, h->stream));
        t += 1;
    }
    h->cur = dst;
    h->jsub = n_sub;
    h->fine_steps += n_sub;
    h->rec_tape = tape;
    h->rec_n = n_sub;
    h->rec_gen = h->gen;
    return HYB_OK;
}

int hyb_lbm_adjoint(hyb_handle *h, int n_sub, const void *tape, const double *lam_in, double *lam_out,
                    double *grad_a, double *grad_b, double *grad_k) {
    if (!h) return HYB_EINVAL;
    if (!tape || tape != h->rec_tape || n_sub != h->rec_n)
        return h->fail(HYB_EINVAL, "the tape and n_sub must be those of the last hyb_lbm_substeps_record");
    if (h->gen != h->rec_gen) return h->fail(HYB_EINVAL, "the handle changed since hyb_lbm_substeps_record");
    if (!lam_in || !lam_out || !grad_a || !grad_b) return h->fail(HYB_EINVAL, "null adjoint argument");
    const size_t fb = h->lay.f_bytes;
    char *base = static_cast<char *>(const_cast<void *>(tape));
    auto slot = [&](int t) { return base + (size_t)t * fb; };
    // the recorded states: f*(0) in the committed buffer, f*(n_sub) in the
    // current one (the handle is unchanged since the record), the others in
    // the tape
    auto state = [&](int t) -> void * {
        if (t == 0) return h->f[h->frozen];
        if (t == n_sub) return h->f[h->cur];
        return slot(t);
    };
    auto uplane = [&](int t) -> const void * {
        if (h->dissolve_on) return nullptr;
        return base + (size_t)(n_sub + 4) * fb + (size_t)(t - 1) * h->lay.u_bytes;
    };
    void *lcur = slot(n_sub + 1), *nu = slot(n_sub + 2), *lnext = slot(n_sub + 3);
    LbmArgs a = h->lbm_args(h->frozen, -1);
    // reversed steps in pairs (one launch each) unless single-step launches
    // were asked for (hyb_set_steps_per_launch(1))
    const bool pairs = h->steps_per_launch >= 2;
    int launches = 0;
    for (int t = n_sub - 1; t >= 0; ++launches) t -= (pairs && t >= 1) ? 2 : 1;
    if (launches == 0) {
        HIP_TRY(h, launch_adjoint_pack(a, h->prec, lam_in, lcur, true, h->stream));
        HIP_TRY(h, launch_adjoint_pack(a, h->prec, lam_out, lcur, false, h->stream));
        return HYB_OK;
    }
    // the first launch reads lam_in in its dense layout and the last writes
    // lam_out in it (no packing passes), unless a single launch would read
    // and write the same array (lam_out may alias lam_in)
    const bool dense_out = launches >= 2 || lam_out != lam_in;
    int k = 0;
    for (int t = n_sub - 1; t >= 0; ++k) {
        const double *din = k == 0 ? lam_in : nullptr;
        double *dout = k == launches - 1 && dense_out ? lam_out : nullptr;
        if (pairs && t >= 1) {
            LbmArgs a1 = a, a2 = a;
            a1.src = state(t);
            a1.lam = (double)(t + 1) / (double)h->eta;
            a1.u_rec = uplane(t + 1);
            a2.src = state(t - 1);
            a2.lam = (double)t / (double)h->eta;
            a2.u_rec = uplane(t);
            HIP_TRY(h, launch_adjoint_step2(a1, a2, h->prec, state(t + 1), state(t), lcur, lnext, grad_a, grad_b,
                                            grad_k, h->stream, nullptr, nullptr, din, dout, false));
            t -= 2;
        } else {
            a.src = state(t);
            a.lam = (double)(t + 1) / (double)h->eta;
            a.u_rec = uplane(t + 1);
            HIP_TRY(h, launch_adjoint_step(a, h->prec, state(t + 1), lcur, nu, lnext, grad_a, grad_b, grad_k,
                                           h->stream, nullptr, din, dout, false));
            t -= 1;
        }
        std::swap(lcur, lnext);
    }
    if (!dense_out) HIP_TRY(h, launch_adjoint_pack(a, h->prec, lam_out, lcur, false, h->stream));
    return HYB_OK;
}

}  // extern "C"

namespace {

// Tape of hyb_step_record: f*(t_n), then eta fine states per pass; three
// adjoint fields; the interface arrays a and b of every pass; dJ/da, dJ/db;
// four padded coarse vectors; dJ/du_fc; one solver result per pass; u of
// every fine step's collision.
struct StepTape {
    size_t states = 0, scratch = 0, bc = 0, gab = 0, coarse = 0, lufc = 0, kres = 0, total = 0;
    size_t u = 0;                   // u of every fine step's collision, eta per pass
    size_t mask = 0, after = 0;     // dissolving solids: flag words before, solid flags after the commit
};

StepTape step_tape_layout(const hyb_handle *h, int passes) {
    StepTape T;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    const size_t fb = h->lay.f_bytes;
    const size_t nslots = 4 * (size_t)(h->N - 1);
    T.states = take((1 + (size_t)passes * h->eta) * fb);
    T.scratch = take(3 * fb);
    T.bc = take((1 + (size_t)passes) * nslots * 8);
    T.gab = take(2 * nslots * 8);
    T.coarse = take(4 * align_up(h->lay.vec_len * 8, kAlign));
    T.lufc = take((size_t)h->lay.n * 8);
    T.kres = take((size_t)passes * sizeof(KrylovResult));
    T.u = take((size_t)passes * h->eta * h->lay.u_bytes);
    if (h->dissolve_ws) {
        const size_t nodes = (size_t)h->N * h->lay.pitch;
        T.mask = take(nodes * 2);
        T.after = take(nodes);
    }
    T.total = off;
    return T;
}

int step_adjoint_supported(hyb_handle *h) {
    if (!h->has_mesh) return h->fail(HYB_EINVAL, "the step adjoint needs a coarse mesh");
    if (h->prec == HYB_FP16S) return h->fail(HYB_EINVAL, "the adjoint supports HYB_FP64 and HYB_FP32 storage");
    if (h->any_neumann) return h->fail(HYB_EINVAL, "the adjoint supports Dirichlet perimeter slots only");
    if (h->wall_on) return h->fail(HYB_EINVAL, "the adjoint supports bounce-back walls only");
    return HYB_OK;
}

}  // namespace

extern "C" {

int hyb_step_adjoint_query(const hyb_handle *h, int passes, size_t *tape_bytes) {
    if (!h || !tape_bytes || passes < 1 || !h->has_mesh) return HYB_EINVAL;
    *tape_bytes = step_tape_layout(h, passes).total;
    return HYB_OK;
}

int hyb_step_record(hyb_handle *h, int passes, void *tape) {
    if (!h) return HYB_EINVAL;
    ++h->gen;
    int rc = step_adjoint_supported(h);
    if (rc != HYB_OK) return rc;
    if (passes < 1) return h->fail(HYB_EINVAL, "passes must be >= 1");
    if (!tape || reinterpret_cast<uintptr_t>(tape) % kAlign) return h->fail(HYB_EINVAL, "tape must be 256-byte aligned");
    const StepTape T = step_tape_layout(h, passes);
    const size_t fb = h->lay.f_bytes;
    const size_t nslots = 4 * (size_t)(h->N - 1);
    char *base = static_cast<char *>(tape);
    // f*(t_n) stays in the committed buffer and the last pass's end state
    // is written straight to the buffer the commit makes current; the other
    // fine states go to the tape
    const int f0 = h->frozen, out = h->spare(-1);
    auto state = [&](int p, int t) -> char * {
        if (t == 0) return static_cast<char *>(h->f[f0]);
        if (p == passes - 1 && t == h->eta) return static_cast<char *>(h->f[out]);
        return base + T.states + (1 + (size_t)p * h->eta + t - 1) * fb;
    };
    // u of fine step t of pass p (t = 1 .. eta; not with dissolving solids,
    // whose reversed steps read the states)
    auto uplane = [&](int p, int t) -> void * {
        if (h->dissolve_ws) return nullptr;
        return base + T.u + ((size_t)p * h->eta + t - 1) * h->lay.u_bytes;
    };
    double *bc = reinterpret_cast<double *>(base + T.bc);
    h->rec_step_tape = nullptr;
    for (int attempt = 0; attempt < 2; ++attempt) {
        h->cur = h->frozen;
        h->jsub = 0;
        h->solved_this_step = false;
        if (h->dissolve_ws)
            HIP_TRY(h, hipMemcpyAsync(base + T.mask, h->mask, (size_t)h->N * h->lay.pitch * 2, hipMemcpyDeviceToDevice,
                                      h->stream));
        for (int p = 0; p < passes; ++p) {
            if ((rc = hyb_interface_exchange(h, HYB_F2C)) != HYB_OK) return rc;
            if ((rc = hyb_coarse_step(h, 200)) != HYB_OK) return rc;
            if ((rc = hyb_interface_exchange(h, HYB_C2F)) != HYB_OK) return rc;
            if (p == 0) HIP_TRY(h, hipMemcpyAsync(bc, h->bc_a, nslots * 8, hipMemcpyDeviceToDevice, h->stream));
            HIP_TRY(h, hipMemcpyAsync(bc + (1 + p) * nslots, h->bc_b, nslots * 8, hipMemcpyDeviceToDevice, h->stream));
            const bool pairs = use_two_step(h);
            for (int t = 1; t <= h->eta;) {
                LbmArgs a = h->lbm_args(h->frozen, -1);
                a.src = state(p, t - 1);
                a.lam = (double)t / (double)h->eta;
                a.u_out = uplane(p, t);
                if (h->dissolve_on) {
                    a.flux = h->flux;
                    a.flux_first = t == 1;
                    h->flux_valid = true;
                }
                if (pairs && t + 1 <= h->eta) {
                    // two fine steps, the state between them kept as well
                    a.mid = state(p, t);
                    a.dst = state(p, t + 1);
                    a.u_out2 = uplane(p, t + 1);
                    a.lam2 = (double)(t + 1) / (double)h->eta;
                    HIP_TRY(h, launch_lbm_step2(a, h->prec, h->stream));
                    t += 2;
                    continue;
                }
                a.dst = state(p, t);
                HIP_TRY(h, launch_lbm_step(a, h->prec, false, h->stream));
                t += 1;
            }
            // the next pass's fine-to-coarse transfer reads the current buffer
            if (p < passes - 1)
                HIP_TRY(h, hipMemcpyAsync(h->f[out], state(p, h->eta), fb, hipMemcpyDeviceToDevice, h->stream));
            h->cur = out;
            h->jsub = h->eta;
            h->fine_steps += h->eta;
        }
        rc = hyb_commit(h);
        if (rc != HYB_ENOCONV || h->solve_budget >= h->solve_cap) break;
        h->last_krylov_iters = h->solve_cap;
    }
    if (rc == HYB_OK) {
        // the solid flags the commit left (the converted nodes are those
        // solid before and fluid after)
        if (h->dissolve_ws)
            HIP_TRY(h, hipMemcpyAsync(base + T.after, h->solid_now, (size_t)h->N * h->lay.pitch,
                                      hipMemcpyDeviceToDevice, h->stream));
        h->rec_step_tape = tape;
        h->rec_step_passes = passes;
        h->rec_step_f0 = f0;
        h->rec_step_out = out;
        h->rec_step_gen = h->gen;
    }
    return rc;
}

int hyb_step_adjoint(hyb_handle *h, const void *tape, const double *lam_f, const double *lam_sub, const double *lam_d,
                     double *lam_f_out, double *lam_d_out, double *grad_k, double *grad_outer) {
    if (!h) return HYB_EINVAL;
    int rc = step_adjoint_supported(h);
    if (rc != HYB_OK) return rc;
    if (!tape || tape != h->rec_step_tape) return h->fail(HYB_EINVAL, "the tape must be that of the last hyb_step_record");
    if (h->gen != h->rec_step_gen) return h->fail(HYB_EINVAL, "the handle changed since hyb_step_record");
    if (!lam_f || !lam_f_out || !lam_d_out) return h->fail(HYB_EINVAL, "null adjoint argument");
    const int passes = h->rec_step_passes;
    const StepTape T = step_tape_layout(h, passes);
    const size_t fb = h->lay.f_bytes;
    const size_t nslots = 4 * (size_t)(h->N - 1);
    char *base = static_cast<char *>(const_cast<void *>(tape));
    auto state = [&](int p, int t) -> char * {
        if (t == 0) return static_cast<char *>(h->f[h->rec_step_f0]);
        if (p == passes - 1 && t == h->eta) return static_cast<char *>(h->f[h->rec_step_out]);
        return base + T.states + (1 + (size_t)p * h->eta + t - 1) * fb;
    };
    auto uplane = [&](int p, int t) -> const void * {
        if (h->dissolve_ws) return nullptr;
        return base + T.u + ((size_t)p * h->eta + t - 1) * h->lay.u_bytes;
    };
    void *lcur = base + T.scratch, *nu = base + T.scratch + fb, *lnext = base + T.scratch + 2 * fb;
    double *bc = reinterpret_cast<double *>(base + T.bc);
    double *ga = reinterpret_cast<double *>(base + T.gab), *gb = ga + nslots;
    const size_t vs = align_up(h->lay.vec_len * 8, kAlign);
    double *lam_dn = reinterpret_cast<double *>(base + T.coarse);
    double *lam_d1 = reinterpret_cast<double *>(base + T.coarse + vs);
    double *rhs_t = reinterpret_cast<double *>(base + T.coarse + 2 * vs);
    double *mu = reinterpret_cast<double *>(base + T.coarse + 3 * vs);
    double *lam_ufc = reinterpret_cast<double *>(base + T.lufc);
    KrylovResult *kr = reinterpret_cast<KrylovResult *>(base + T.kres);
    LbmArgs a = h->lbm_args(h->frozen, -1);
    const bool dissolving = h->dissolve_ws;
    if (dissolving) a.mask = reinterpret_cast<const uint16_t *>(base + T.mask);   // the step's geometry
    // the first reversed launch reads lam_f in its dense layout (no packing
    // pass) unless the conversion's transpose works on it first or lam_f_out
    // (cleared below) aliases it
    const bool dense_in = !dissolving && lam_f_out != lam_f;
    if (!dense_in) HIP_TRY(h, launch_adjoint_pack(a, h->prec, lam_f, lcur, true, h->stream));
    if (dissolving) {
        // the commit's conversion, transposed (nu is free until the first reversed fine step)
        HIP_TRY(h, launch_conversion_transpose(a, h->prec, reinterpret_cast<const uint8_t *>(base + T.after),
                                               state(passes - 1, h->eta), lcur, static_cast<double *>(nu), grad_k,
                                               h->stream));
    }
    // the cotangent of the committed pass's intermediate fine states, in the
    // storage layout (nu is free from here on: the fused reversed steps keep
    // their nu on chip)
    const void *inj = nullptr;
    if (lam_sub) {
        HIP_TRY(h, launch_adjoint_pack(a, h->prec, lam_sub, nu, true, h->stream));
        inj = nu;
    }
    // lam_f_out: the last reversed launch of the first pass reversed writes
    // it whole (zeros at solid nodes), the other passes and the transfer add
    // the padded coarse vectors keep a zero halo (stencils read it)
    HIP_TRY(h, hipMemsetAsync(base + T.coarse, 0, 4 * vs, h->stream));
    CoarseDev ct = h->cd;
    ct.AP = h->apt;
    const int budget = std::min(200, std::max(16, 2 * h->last_krylov_iters + 6));
    for (int p = passes - 1; p >= 0; --p) {
        // fine steps of pass p, reversed (interface values of the pass)
        HIP_TRY(h, hipMemsetAsync(ga, 0, 2 * nslots * 8, h->stream));
        a.bc_a = bc;
        a.bc_b = bc + (1 + p) * nslots;
        // the committed pass's intermediate states t = 1 .. eta-1 take the
        // substep cotangent (state eta takes lam_f, state 0 belongs to the
        // previous coarse step)
        const void *inj_p = p == passes - 1 ? inj : nullptr;
        int launches = 0;
        for (int t = h->eta; t >= 1; ++launches) t -= (h->steps_per_launch >= 2 && t >= 2) ? 2 : 1;
        int k = 0;
        for (int t = h->eta; t >= 1; ++k) {
            // the pass's last launch adds its output to lam_f_out directly
            const double *din = dense_in && p == passes - 1 && k == 0 ? lam_f : nullptr;
            double *dout = k == launches - 1 ? lam_f_out : nullptr;
            const bool add = p != passes - 1;
            if (h->steps_per_launch >= 2 && t >= 2) {
                // steps t and t-1 reversed in one launch
                LbmArgs a1 = a, a2 = a;
                a1.src = state(p, t - 1);
                a1.lam = (double)t / (double)h->eta;
                a1.u_rec = uplane(p, t);
                a2.src = state(p, t - 2);
                a2.lam = (double)(t - 1) / (double)h->eta;
                a2.u_rec = uplane(p, t - 1);
                HIP_TRY(h, launch_adjoint_step2(a1, a2, h->prec, state(p, t), state(p, t - 1), lcur, lnext, ga, gb,
                                                grad_k, h->stream, inj_p, t - 2 >= 1 ? inj_p : nullptr, din, dout,
                                                add));
                t -= 2;
            } else {
                a.src = state(p, t - 1);
                a.lam = (double)t / (double)h->eta;
                a.u_rec = uplane(p, t);
                HIP_TRY(h, launch_adjoint_step(a, h->prec, state(p, t), lcur, nu, lnext, ga, gb, grad_k, h->stream,
                                               t - 1 >= 1 ? inj_p : nullptr, din, dout, add));
                t -= 1;
            }
            std::swap(lcur, lnext);
        }
        // coarse-to-fine, coarse solve and right-hand side, transposed
        HIP_TRY(h, launch_c2f_transpose(h->cd, h->c2fT_ptr, h->c2fT_slot, h->c2fT_w, ga, gb,
                                        p == passes - 1 ? lam_d : nullptr, lam_dn, lam_d1, h->stream));
        HIP_TRY(h, launch_coarse_stencil(h->cd, h->pt, kSpaiW, lam_d1, rhs_t, h->stream));
        ct.result = kr + p;
        HIP_TRY(h, launch_coarse_solve_given(ct, rhs_t, mu, budget, 200, 1e-14, h->stream));
        HIP_TRY(h, launch_coarse_rhs_transpose(h->cd, h->fc_row, h->nfc, mu, lam_dn, lam_ufc, grad_outer, h->stream));
        // fine-to-coarse transposed onto the state the pass's transfer read
        const void *read = p == 0 ? state(0, 0) : state(p - 1, h->eta);
        if (p > 0) HIP_TRY(h, hipMemsetAsync(lcur, 0, fb, h->stream));
        void *to_pitched = p == 0 ? nullptr : lcur;
        double *to_dense = p == 0 ? lam_f_out : nullptr;
        if (dissolving)
            HIP_TRY(h, launch_f2c_dynamic_transpose(a, h->prec, h->f2cD_node, h->f2cD_ptr, h->f2cD_c, h->f2cD_m,
                                                    h->f2cD_n, h->fcr_idx, h->fcr_w, lam_ufc, read, to_pitched,
                                                    to_dense, grad_k, h->stream));
        else
            HIP_TRY(h, launch_f2c_transpose(a, h->prec, h->f2cT_node, h->f2cT_ptr, h->f2cT_c, h->f2cT_w, h->f2cT_n,
                                            lam_ufc, read, to_pitched, to_dense, grad_k, h->stream));
    }
    HIP_TRY(h, launch_coarse_repad(h->cd, lam_dn, lam_d_out, true, h->stream));
    std::vector<KrylovResult> res(passes);
    HIP_TRY(h, hipMemcpyAsync(res.data(), kr, passes * sizeof(KrylovResult), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int p = 0; p < passes; ++p)
        if (!res[p].converged) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "transposed coarse solve of pass %d did not converge (%d iterations, relres %.3e)",
                          p, res[p].iters, res[p].relres);
            return h->fail(HYB_ENOCONV, buf);
        }
    return HYB_OK;
}

}  // extern "C"

namespace {

}  // namespace

extern "C" {

int hyb_set_steps_per_launch(hyb_handle *h, int steps) {
    if (!h) return HYB_EINVAL;
    if (steps < 1 || steps > 5) return h->fail(HYB_EINVAL, "steps per launch must be 1 to 5");
    h->steps_per_launch = steps;
    // the launch plan sets the overlap depths available: tune again
    h->tune_idx = 0;
    h->tuned_depth = -1;
    h->tune_ms.clear();
    return HYB_OK;
}

int hyb_kernel_timing(hyb_handle *h, int enable) {
    if (!h) return HYB_EINVAL;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, h->drain_events());
    h->timing = enable != 0;
    h->timed_ms = 0.0;
    h->timed_launches = 0;
    return HYB_OK;
}

int hyb_kernel_time(hyb_handle *h, double *total_ms, int64_t *launches) {
    if (!h) return HYB_EINVAL;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, h->drain_events());
    if (total_ms) *total_ms = h->timed_ms;
    if (launches) *launches = h->timed_launches;
    h->timed_ms = 0.0;
    h->timed_launches = 0;
    return HYB_OK;
}

int hyb_layout(const hyb_handle *h, size_t *pitch, size_t *plane) {
    if (!h) return HYB_EINVAL;
    if (pitch) *pitch = (size_t)h->lay.pitch;
    if (plane) *plane = (size_t)h->lay.plane;
    return HYB_OK;
}

void hyb_destroy(hyb_handle *h) { delete h; }

const char *hyb_last_error(const hyb_handle *h) { return h ? h->err.c_str() : "null handle"; }

int hyb_set_wall_normals(hyb_handle *h, const float *normals) {
    if (!h) return HYB_EINVAL;
    ++h->gen;
    if (!h->wall_ws) return h->fail(HYB_EINVAL, "the handle was created without the wall closure");
    if (h->jsub != 0 || h->cur != h->frozen)
        return h->fail(HYB_EINVAL, "set the wall closure between coarse steps (fine steps are pending)");
    if (!normals) {
        h->wall_on = false;
        return HYB_OK;
    }
    if (h->dissolve_on) return h->fail(HYB_EINVAL, "dissolving solids need bounce-back walls");
    if (refresh_solid_host(h) != hipSuccess) return h->fail(HYB_EHIP, "could not read the solid flags");
    const int N = h->N, P = h->lay.pitch;
    const size_t NN = (size_t)N * N;
    std::vector<float> nx((size_t)N * P, 0.f), ny((size_t)N * P, 0.f);
    auto solid = [&](int i, int j) { return h->solid_host[(size_t)j * N + i] != 0; };
    for (int j = 1; j < N - 1; ++j)
        for (int i = 1; i < N - 1; ++i) {
            if (solid(i, j)) continue;
            bool wall = false;
            for (int q = 1; q < kQ; ++q) wall = wall || solid(i - kCx[q], j - kCy[q]);
            if (!wall) continue;
            const float x = normals[(size_t)j * N + i], y = normals[NN + (size_t)j * N + i];
            const double len = std::sqrt((double)x * x + (double)y * y);
            if (!std::isfinite(len) || std::fabs(len - 1.0) > 1e-3)
                return h->fail(HYB_EINVAL, "every fluid node next to a solid needs a unit wall normal");
            nx[(size_t)j * P + i] = x;
            ny[(size_t)j * P + i] = y;
        }
    HIP_TRY(h, hipMemcpyAsync(h->wall_nx, nx.data(), nx.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->wall_ny, ny.data(), ny.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->wall_on = true;
    // the sweeps change (single steps, no overlap), so the depth is tuned again
    h->tune_idx = 0;
    h->tuned_depth = -1;
    h->tune_ms.clear();
    return HYB_OK;
}

int hyb_set_dissolution(hyb_handle *h, double kappa_s, double c_sat, const double *mass) {
    if (!h) return HYB_EINVAL;
    ++h->gen;
    if (!h->dissolve_ws) return h->fail(HYB_EINVAL, "the handle was created without dissolution");
    if (!(kappa_s >= 0.0 && kappa_s <= 1.0)) return h->fail(HYB_EINVAL, "kappa_s must lie in [0, 1]");
    if (!std::isfinite(c_sat)) return h->fail(HYB_EINVAL, "c_sat must be finite");
    if (h->jsub != 0 || h->cur != h->frozen)
        return h->fail(HYB_EINVAL, "set the dissolution between coarse steps (fine steps are pending)");
    if (h->wall_on && kappa_s > 0.0)
        return h->fail(HYB_EINVAL, "dissolving solids need bounce-back walls (the wall closure is on)");
    if (refresh_solid_host(h) != hipSuccess) return h->fail(HYB_EHIP, "could not read the solid flags");
    if (mass) {
        const int N = h->N, P = h->lay.pitch;
        std::vector<double> mp((size_t)N * P, 0.0);
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i)
                if (h->solid_host[(size_t)j * N + i]) mp[(size_t)j * P + i] = mass[(size_t)j * N + i];
        HIP_TRY(h, hipMemcpyAsync(h->mass, mp.data(), mp.size() * 8, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    h->kappa_s = kappa_s;
    h->c_sat = c_sat;
    h->dissolve_on = kappa_s > 0.0;
    h->flux_valid = false;
    // the sweeps change (whole-patch launches with the reaction), so the
    // overlap depth is tuned again
    h->tune_idx = 0;
    h->tuned_depth = -1;
    h->tune_ms.clear();
    return HYB_OK;
}

}  // extern "C"

namespace {

// Checkpoint layout (device bytes, 256-byte aligned parts): the committed
// populations (storage format), the coarse solutions d(t_n) and d(t_{n-1})
// (padded), and with dissolving solids the flag words, solid flags and
// masses.
struct CkptLayout {
    size_t f = 0, xn = 0, xprev = 0, mask = 0, solid = 0, mass = 0, total = 0;
};

CkptLayout ckpt_layout(const hyb_handle *h) {
    CkptLayout C;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    const size_t nodes = (size_t)h->N * h->lay.pitch;
    C.f = take(h->lay.f_bytes);
    if (h->has_mesh) {
        C.xn = take(h->lay.vec_len * 8);
        C.xprev = take(h->lay.vec_len * 8);
    }
    if (h->dissolve_ws) {
        C.mask = take(nodes * 2);
        C.solid = take(nodes);
        C.mass = take(nodes * 8);
    }
    C.total = off;
    return C;
}

}  // namespace

extern "C" {

int hyb_checkpoint_query(const hyb_handle *h, size_t *bytes) {
    if (!h || !bytes) return HYB_EINVAL;
    *bytes = ckpt_layout(h).total;
    return HYB_OK;
}

int hyb_checkpoint_save(hyb_handle *h, void *ckpt) {
    if (!h || !ckpt || reinterpret_cast<uintptr_t>(ckpt) % kAlign) return HYB_EINVAL;
    if (h->jsub != 0 || h->cur != h->frozen)
        return h->fail(HYB_EINVAL, "checkpoint between coarse steps (fine steps are pending)");
    const CkptLayout C = ckpt_layout(h);
    char *b = static_cast<char *>(ckpt);
    const size_t nodes = (size_t)h->N * h->lay.pitch;
    auto cp = [&](void *dst, const void *src, size_t n) {
        return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, h->stream);
    };
    HIP_TRY(h, cp(b + C.f, h->f[h->frozen], h->lay.f_bytes));
    if (h->has_mesh) {
        HIP_TRY(h, cp(b + C.xn, h->cd.xn, h->lay.vec_len * 8));
        HIP_TRY(h, cp(b + C.xprev, h->cd.xprev, h->lay.vec_len * 8));
    }
    if (h->dissolve_ws) {
        HIP_TRY(h, cp(b + C.mask, h->mask, nodes * 2));
        HIP_TRY(h, cp(b + C.solid, h->solid_now, nodes));
        HIP_TRY(h, cp(b + C.mass, h->mass, nodes * 8));
    }
    return HYB_OK;
}

int hyb_checkpoint_load(hyb_handle *h, const void *ckpt) {
    if (!h || !ckpt || reinterpret_cast<uintptr_t>(ckpt) % kAlign) return HYB_EINVAL;
    ++h->gen;
    const CkptLayout C = ckpt_layout(h);
    const char *b = static_cast<const char *>(ckpt);
    const size_t nodes = (size_t)h->N * h->lay.pitch;
    auto cp = [&](void *dst, const void *src, size_t n) {
        return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, h->stream);
    };
    HIP_TRY(h, cp(h->f[h->frozen], b + C.f, h->lay.f_bytes));
    if (h->has_mesh) {
        HIP_TRY(h, cp(h->cd.xn, b + C.xn, h->lay.vec_len * 8));
        HIP_TRY(h, cp(h->cd.xprev, b + C.xprev, h->lay.vec_len * 8));
    }
    if (h->dissolve_ws) {
        HIP_TRY(h, cp(h->mask, b + C.mask, nodes * 2));
        HIP_TRY(h, cp(h->solid_now, b + C.solid, nodes));
        HIP_TRY(h, cp(h->mass, b + C.mass, nodes * 8));
        h->solid_host_stale = true;
        h->flux_valid = false;
    }
    h->cur = h->frozen;
    h->jsub = 0;
    h->solved_this_step = false;
    return HYB_OK;
}

int hyb_set_solids(hyb_handle *h, const uint8_t *solid, const double *mass) {
    if (!h || !solid || !mass) return HYB_EINVAL;
    ++h->gen;
    if (!h->dissolve_ws) return h->fail(HYB_EINVAL, "the handle was created without dissolution");
    if (h->jsub != 0 || h->cur != h->frozen)
        return h->fail(HYB_EINVAL, "set the solids between coarse steps (fine steps are pending)");
    const int N = h->N, P = h->lay.pitch;
    for (size_t n = 0; n < (size_t)N * N; ++n)
        if (solid[n] && !h->solid_init[n])
            return h->fail(HYB_EINVAL, "only nodes that were solid at creation can be solid");
    std::vector<uint8_t> sp((size_t)N * P, 0);
    std::vector<double> mp((size_t)N * P, 0.0);
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            const size_t n = (size_t)j * N + i;
            sp[(size_t)j * P + i] = solid[n] ? 1 : 0;
            mp[(size_t)j * P + i] = solid[n] ? mass[n] : 0.0;
        }
    HIP_TRY(h, hipMemcpyAsync(h->solid_now, sp.data(), sp.size(), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->mass, mp.data(), mp.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, launch_mask_rebuild(N, P, h->solid_now, h->mask, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (size_t n = 0; n < (size_t)N * N; ++n) h->solid_host[n] = solid[n] ? 1 : 0;
    h->solid_host_stale = false;
    h->flux_valid = false;
    return HYB_OK;
}

int hyb_dissolution_state(hyb_handle *h, uint8_t *solid, double *mass, int64_t *converted) {
    if (!h) return HYB_EINVAL;
    if (!h->dissolve_ws) return h->fail(HYB_EINVAL, "the handle was created without dissolution");
    if (refresh_solid_host(h) != hipSuccess) return h->fail(HYB_EHIP, "could not read the solid flags");
    const int N = h->N, P = h->lay.pitch;
    if (solid) std::memcpy(solid, h->solid_host.data(), (size_t)N * N);
    if (mass) {
        std::vector<double> mp((size_t)N * P);
        HIP_TRY(h, hipMemcpyAsync(mp.data(), h->mass, mp.size() * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i)
                mass[(size_t)j * N + i] = h->solid_host[(size_t)j * N + i] ? mp[(size_t)j * P + i] : 0.0;
    }
    if (converted) {
        // fluid never turns solid, so the solids gone since creation are the conversions
        int64_t c = 0;
        for (size_t n = 0; n < (size_t)N * N; ++n) c += (int64_t)h->solid_init[n] - (int64_t)h->solid_host[n];
        *converted = c;
    }
    return HYB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Several fine patches around one coarse subdomain (Algorithm 2, Sec. 6.3):
// the patches are lattice-only handles (their perimeter values a, b are the
// interface arrays of hyb_set_boundary); the group owns the coarse operator,
// whose Dirichlet rows are the outer edge and every patch's Gamma_{f->c},
// and per patch the two transfer lists.
// ---------------------------------------------------------------------------

namespace {

struct GroupLayout {
    size_t A9 = 0, B9 = 0, AP = 0, P = 0, dkind = 0, vec = 0, partials = 0, state = 0, kres = 0, ufc = 0;
    std::vector<size_t> c2f_idx, c2f_w, fc_idx, fc_w;
    size_t total = 0;
    int n = 0, S = 0, grid = 0;
    size_t vec_len = 0;
};

GroupLayout group_layout(int M, const std::vector<int> &patch_N) {
    GroupLayout G;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    G.n = (M + 1) * (M + 1);
    G.S = M + 1 + 2 * kCoarseHalo;
    G.grid = coarse_grid(G.n);
    G.vec_len = (size_t)G.S * G.S;
    G.A9 = take((size_t)G.n * 9 * 8);
    G.B9 = take((size_t)G.n * 9 * 8);
    G.AP = take((size_t)G.n * kApW * kApW * 8);
    G.P = take((size_t)G.n * kSpaiW * kSpaiW * 8);
    G.dkind = take((size_t)G.n * 4);
    G.vec = take(12 * align_up(G.vec_len * 8, kAlign));
    G.partials = take((size_t)4 * kPartialValues * coarse_grid8(G.n) * 8);
    G.state = take(sizeof(KrylovState));
    G.kres = take(sizeof(KrylovResult));
    G.ufc = take((size_t)G.n * 8);
    for (int N : patch_N) {
        const size_t nslots = 4 * (size_t)(N - 1);
        G.c2f_idx.push_back(take(nslots * 4 * 4));
        G.c2f_w.push_back(take(nslots * 4 * 8));
        G.fc_idx.push_back(take((size_t)G.n * 4 * 4));
        G.fc_w.push_back(take((size_t)G.n * 4 * 8));
    }
    G.total = off;
    return G;
}

}  // namespace

struct hyb_group {
    std::string err;
    std::vector<hyb_handle *> patches;
    std::vector<int> nfc, off;          // Gamma_{f->c} nodes of each patch and their run's start
    std::vector<int *> c2f_idx, fc_idx;
    std::vector<double *> c2f_w, fc_w;
    GroupLayout lay;
    CoarseDev cd{};
    double *ufc = nullptr;
    KrylovResult *kres = nullptr;
    hipStream_t stream = nullptr;
    int M = 0, eta = 1;
    bool solved = false;
    int last_iters = 8, budget = 0, cap = 0;
    int fail(int code, const std::string &msg) {
        err = msg;
        return code;
    }
};

extern "C" {

int hyb_group_query(const hyb_mesh *mesh, int n, const hyb_lattice *lattices, size_t *ws_bytes) {
    if (!mesh || mesh->M < 2 || n < 1 || !lattices || !ws_bytes) return HYB_EINVAL;
    std::vector<int> Ns;
    for (int p = 0; p < n; ++p) {
        if (lattices[p].N < 3) return HYB_EINVAL;
        Ns.push_back(lattices[p].N);
    }
    *ws_bytes = group_layout(mesh->M, Ns).total;
    return HYB_OK;
}

int hyb_group_create(const hyb_mesh *mesh, int n, hyb_handle *const *patches, double D, const double *vcoarse,
                     double k, void *workspace, void *stream, hyb_group **out) {
    if (!out) return HYB_EINVAL;
    *out = nullptr;
    if (!mesh || mesh->M < 2 || !(mesh->L > 0.0) || !mesh->d0 || mesh->overlap_elems < 1 || n < 1 || !patches ||
        !vcoarse || !(D > 0.0) || !(k >= 0.0 && k < 1.0) || !workspace ||
        reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return HYB_EINVAL;
    std::vector<PatchGeom> geo;
    std::vector<int> Ns;
    for (int p = 0; p < n; ++p) {
        const hyb_handle *h = patches[p];
        if (!h || h->has_mesh || h->kinds_set || h->dissolve_ws || h->eta != patches[0]->eta) {
            std::fprintf(stderr, "hyb_group_create: patches must be lattice-only handles with Dirichlet perimeters, "
                                 "fixed solids and one eta\n");
            return HYB_EINVAL;
        }
        if (h->x0 < 0 || h->y0 < 0 || h->x0 + (h->N - 1) > mesh->L || h->y0 + (h->N - 1) > mesh->L) {
            std::fprintf(stderr, "hyb_group_create: patch %d lies outside the coarse domain\n", p);
            return HYB_EINVAL;
        }
        geo.push_back(PatchGeom{h->N, h->x0, h->y0, h->solid_host.data(), h->lay.pitch});
        Ns.push_back(h->N);
    }
    CoarseHost ch;
    std::vector<CoarseHost> more;
    const std::string msg = build_coarse(mesh->M, mesh->L, D, k, (double)patches[0]->eta, mesh->supg, vcoarse,
                                         mesh->overlap_elems, geo, ch, &more, mesh->outer_natural);
    if (!msg.empty()) {
        std::fprintf(stderr, "hyb_group_create: %s\n", msg.c_str());
        return HYB_EINVAL;
    }
    hyb_group *g = new hyb_group();
    g->lay = group_layout(mesh->M, Ns);
    const GroupLayout &L = g->lay;
    g->stream = static_cast<hipStream_t>(stream);
    g->M = mesh->M;
    g->eta = patches[0]->eta;
    char *ws = static_cast<char *>(workspace);
    hipStream_t st = g->stream;
    auto bail = [&](hipError_t e, const char *what) {
        std::fprintf(stderr, "hyb_group_create: %s: %s\n", what, hipGetErrorString(e));
        delete g;
        return HYB_EHIP;
    };
#define GROUP_TRY(call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return bail(e_, #call);     \
    } while (0)
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    GROUP_TRY(hipMemsetAsync(ws, 0, L.total, st));
    int off = 0;
    for (int p = 0; p < n; ++p) {
        const CoarseHost &c = p == 0 ? ch : more[p - 1];
        g->patches.push_back(patches[p]);
        g->nfc.push_back((int)c.fc_nodes.size());
        g->off.push_back(off);
        off += (int)c.fc_nodes.size();
        g->c2f_idx.push_back(reinterpret_cast<int *>(ws + L.c2f_idx[p]));
        g->c2f_w.push_back(reinterpret_cast<double *>(ws + L.c2f_w[p]));
        g->fc_idx.push_back(reinterpret_cast<int *>(ws + L.fc_idx[p]));
        g->fc_w.push_back(reinterpret_cast<double *>(ws + L.fc_w[p]));
        GROUP_TRY(up(g->c2f_idx[p], c.c2f_idx.data(), c.c2f_idx.size() * 4));
        GROUP_TRY(up(g->c2f_w[p], c.c2f_w.data(), c.c2f_w.size() * 8));
        if (!c.fc_nodes.empty()) {
            GROUP_TRY(up(g->fc_idx[p], c.fc_idx.data(), c.fc_idx.size() * 4));
            GROUP_TRY(up(g->fc_w[p], c.fc_w.data(), c.fc_w.size() * 8));
        }
    }
    CoarseDev &c = g->cd;
    c.M = mesh->M;
    c.n = L.n;
    c.S = L.S;
    c.grid = L.grid;
    c.grid8 = coarse_grid8(L.n);
    c.pstride = c.grid8;
    c.A9 = reinterpret_cast<const double *>(ws + L.A9);
    c.B9 = reinterpret_cast<const double *>(ws + L.B9);
    c.AP = reinterpret_cast<const double *>(ws + L.AP);
    c.P = reinterpret_cast<const double *>(ws + L.P);
    c.dkind = reinterpret_cast<const int *>(ws + L.dkind);
    c.outer_value = mesh->outer_value;
    g->ufc = reinterpret_cast<double *>(ws + L.ufc);
    c.ufc = g->ufc;
    const size_t vstride = align_up(L.vec_len * 8, kAlign);
    double *vec[12];
    for (int v = 0; v < 12; ++v) vec[v] = reinterpret_cast<double *>(ws + L.vec + v * vstride);
    c.xn = vec[0];
    c.x1 = vec[1];
    c.r = vec[2];
    c.rh = vec[3];
    c.p = vec[4];
    c.v = vec[5];
    c.s = vec[6];
    c.t = vec[7];
    c.y = vec[8];
    c.w = vec[9];
    c.z = vec[10];
    c.xprev = vec[11];
    c.partials = reinterpret_cast<double *>(ws + L.partials);
    c.state = reinterpret_cast<KrylovState *>(ws + L.state);
    g->kres = reinterpret_cast<KrylovResult *>(ws + L.kres);
    c.result = g->kres;
    const std::vector<double> A9t = offset_major(ch.A9, L.n, 9), B9t = offset_major(ch.B9, L.n, 9);
    const std::vector<double> Pt = offset_major(ch.P, L.n, kSpaiW * kSpaiW);
    GROUP_TRY(up((void *)c.A9, A9t.data(), A9t.size() * 8));
    GROUP_TRY(up((void *)c.B9, B9t.data(), B9t.size() * 8));
    GROUP_TRY(up((void *)c.AP, ch.AP.data(), ch.AP.size() * 8));
    GROUP_TRY(up((void *)c.P, Pt.data(), Pt.size() * 8));
    GROUP_TRY(up((void *)c.dkind, ch.dkind.data(), ch.dkind.size() * 4));
    std::vector<double> xp(L.vec_len, 0.0);
    const int m1 = mesh->M + 1;
    for (int l = 0; l < m1; ++l)
        for (int kk = 0; kk < m1; ++kk) xp[(size_t)(l + kCoarseHalo) * L.S + kk + kCoarseHalo] = mesh->d0[l * m1 + kk];
    GROUP_TRY(up(c.xn, xp.data(), xp.size() * 8));
    GROUP_TRY(up(c.x1, xp.data(), xp.size() * 8));
    GROUP_TRY(up(c.xprev, xp.data(), xp.size() * 8));
    GROUP_TRY(hipStreamSynchronize(st));
#undef GROUP_TRY
    *out = g;
    return HYB_OK;
}

int hyb_group_step(hyb_group *g, int max_schwarz) {
    if (!g) return HYB_EINVAL;
    if (max_schwarz < 1) return g->fail(HYB_EINVAL, "max_schwarz must be >= 1");
    for (hyb_handle *h : g->patches)
        if (h->stream != g->stream) return g->fail(HYB_EINVAL, "the patches must use the group's stream");
    auto hip = [&](hipError_t e, const char *what) {
        return e == hipSuccess ? HYB_OK : g->fail(HYB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    };
    int rc = HYB_OK;
    const int np = (int)g->patches.size();
    for (int attempt = 0; attempt < 2; ++attempt) {
        for (hyb_handle *h : g->patches) {
            h->cur = h->frozen;
            h->jsub = 0;
        }
        g->solved = false;
        for (int it = 0; it < max_schwarz; ++it) {
            // every patch's transfer (its state at t_n, then its last result)
            for (int p = 0; p < np; ++p) {
                hyb_handle *h = g->patches[p];
                LbmArgs a = h->lbm_args(h->cur, -1);
                if ((rc = hip(launch_f2c(a, g->fc_idx[p], g->fc_w[p], g->nfc[p], g->ufc + g->off[p], h->prec,
                                         g->stream), "fine-to-coarse")) != HYB_OK)
                    return rc;
            }
            // the shared coarse step
            if (!g->solved && (rc = hip(launch_coarse_extrapolate(g->cd, g->stream), "extrapolate")) != HYB_OK)
                return rc;
            g->budget = std::min(200, std::max(4, g->last_iters + 2));
            g->cap = 200;
            if ((rc = hip(launch_coarse_rhs(g->cd, g->cd.x1, g->stream), "coarse rhs")) != HYB_OK) return rc;
            if ((rc = hip(launch_coarse_solve(g->cd, g->cd.x1, g->budget, 200, 1e-14, g->stream), "coarse solve")) !=
                HYB_OK)
                return rc;
            g->solved = true;
            // every patch's perimeter values and fine steps
            for (int p = 0; p < np; ++p) {
                hyb_handle *h = g->patches[p];
                if ((rc = hip(launch_c2f(g->c2f_idx[p], g->c2f_w[p], 4 * (h->N - 1), g->cd.xn, g->cd.x1, h->bc_a,
                                         h->bc_b, g->stream), "coarse-to-fine")) != HYB_OK)
                    return rc;
            }
            for (hyb_handle *h : g->patches)
                if ((rc = substeps_impl(h, g->eta, 1, -1, 0)) != HYB_OK) return g->fail(rc, h->err);
        }
        KrylovResult kr{};
        if ((rc = hip(hipMemcpyAsync(&kr, g->kres, sizeof(kr), hipMemcpyDeviceToHost, g->stream), "result")) != HYB_OK)
            return rc;
        if ((rc = hip(hipStreamSynchronize(g->stream), "synchronise")) != HYB_OK) return rc;
        g->last_iters = kr.iters;
        if (kr.converged) break;
        if (g->budget >= g->cap || attempt == 1) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "coarse solve did not converge (%d iterations, relres %.3e)", kr.iters,
                          kr.relres);
            return g->fail(HYB_ENOCONV, buf);
        }
        g->last_iters = g->cap;
    }
    // commit every patch (non-finite checks), then the coarse state
    for (hyb_handle *h : g->patches)
        if ((rc = hyb_commit(h)) != HYB_OK) return g->fail(rc, h->err);
    double *old_prev = g->cd.xprev;
    g->cd.xprev = g->cd.xn;
    g->cd.xn = g->cd.x1;
    g->cd.x1 = old_prev;
    g->solved = false;
    return HYB_OK;
}

int hyb_group_coarse(hyb_group *g, double *out, int out_is_device) {
    if (!g || !out) return HYB_EINVAL;
    const int m1 = g->M + 1;
    const size_t rowb = (size_t)m1 * 8;
    const hipError_t e = hipMemcpy2DAsync(out, rowb, g->cd.xn + (size_t)kCoarseHalo * g->cd.S + kCoarseHalo,
                                          (size_t)g->cd.S * 8, rowb, m1,
                                          out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream);
    if (e != hipSuccess || hipStreamSynchronize(g->stream) != hipSuccess) return g->fail(HYB_EHIP, "coarse readout");
    return HYB_OK;
}

void hyb_group_destroy(hyb_group *g) { delete g; }

const char *hyb_group_last_error(const hyb_group *g) { return g ? g->err.c_str() : "null group"; }

}  // extern "C"
