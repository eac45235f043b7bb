// Host side of the C ABI declared in include/nco.h: lattice objects, argument
// checking, device buffers, the A/B population swap and kernel dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/nco.h"
#include "kernels.h"

using namespace nco;

namespace nco {
int spectrum_bins(int n);
}

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? NCO_E_OOM : NCO_E_HIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

size_t store_bytes(int storage) {
    switch (storage) {
        case NCO_F32: return 4;
        case NCO_F16_DEV: return 2;
        case NCO_BF16_DEV: return 2;
        case NCO_F64: return 8;
        default: return 0;
    }
}

bool width_ok(int w) { return w == 8 || w == 16 || w == 20 || w == 32; }

size_t n_params_for(int width) { return (size_t)width * (27 + width + 4) + 2 * (size_t)width + 4; }
size_t n_params_depth(int width, int depth) {
    return n_params_for(width) + (depth == 3 ? (size_t)width * width + width : 0);
}

// Parameters of a width-W network (order W1, b1, W2, b2, [W2b, b2b,] W3, b3,
// each W [in][out]) zero-padded to width P: a padded hidden unit has zero
// weights in and out and a zero bias, so it adds exactly nothing.
std::vector<float> pad_params(const float* p, int W, int depth, int P) {
    std::vector<float> out(n_params_depth(P, depth), 0.0f);
    const float* s = p;
    float* d = out.data();
    for (int k = 0; k < 27; ++k)
        for (int h = 0; h < W; ++h) d[k * P + h] = s[k * W + h];
    s += 27 * W;
    d += 27 * P;
    for (int h = 0; h < W; ++h) d[h] = s[h];
    s += W;
    d += P;
    for (int layer = 1; layer < depth; ++layer) {
        for (int i = 0; i < W; ++i)
            for (int o = 0; o < W; ++o) d[i * P + o] = s[i * W + o];
        s += W * W;
        d += P * P;
        for (int o = 0; o < W; ++o) d[o] = s[o];
        s += W;
        d += P;
    }
    for (int i = 0; i < W; ++i)
        for (int n = 0; n < 4; ++n) d[i * 4 + n] = s[i * 4 + n];
    s += 4 * W;
    d += 4 * P;
    for (int n = 0; n < 4; ++n) d[n] = s[n];
    return out;
}

// Depth-3 gradient from the vector-unit adjoint's row layout at width P
// (W1, b1, W2, b2, W3, b3, then W2b, b2b) to the parameter order at width W
// (W1, b1, W2, b2, W2b, b2b, W3, b3), dropping the padded units.
void unpad_grad3(const double* g, int P, int W, double* out) {
    const double* gW1 = g;
    const double* gb1 = gW1 + 27 * P;
    const double* gW2 = gb1 + P;
    const double* gb2 = gW2 + P * P;
    const double* gW3 = gb2 + P;
    const double* gb3 = gW3 + 4 * P;
    const double* gW2b = gb3 + 4;
    const double* gb2b = gW2b + P * P;
    double* d = out;
    for (int k = 0; k < 27; ++k)
        for (int h = 0; h < W; ++h) *d++ = gW1[k * P + h];
    for (int h = 0; h < W; ++h) *d++ = gb1[h];
    for (int i = 0; i < W; ++i)
        for (int o = 0; o < W; ++o) *d++ = gW2[i * P + o];
    for (int o = 0; o < W; ++o) *d++ = gb2[o];
    for (int i = 0; i < W; ++i)
        for (int o = 0; o < W; ++o) *d++ = gW2b[i * P + o];
    for (int o = 0; o < W; ++o) *d++ = gb2b[o];
    for (int i = 0; i < W; ++i)
        for (int n = 0; n < 4; ++n) *d++ = gW3[i * 4 + n];
    for (int n = 0; n < 4; ++n) *d++ = gb3[n];
}

// Paper row of a Hermite multi-index (inverse of row_tensor).
int row_of_tensor(int t) {
    for (int k = 0; k < 27; ++k)
        if (row_tensor(k) == t) return k;
    return -1;
}

// The 48 elements of O_h as (axis permutation, axis signs): (R c)_r =
// s_r c_{perm_r}.  For each element and each row k of M, the group action on
// the moments is m^(g)_k = sign * m_{src}: with h_n(-x) = (-1)^n h_n(x), the
// row with multi-index n_k evaluated at R c is the row with multi-index n'
// (n'_{perm_r} = n_{k,r}) times prod_r s_r^{n_{k,r}}.
struct GroupAction {
    int src[48][27];
    float sign[48][27];
};

GroupAction build_group_action() {
    GroupAction G;
    int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int g = 0;
    for (auto& p : perms)
        for (int sm = 0; sm < 8; ++sm) {
            const int s[3] = {(sm & 1) ? -1 : 1, (sm & 2) ? -1 : 1, (sm & 4) ? -1 : 1};
            for (int k = 0; k < 27; ++k) {
                const int t = row_tensor(k);
                const int n[3] = {t % 3, (t / 3) % 3, t / 9};
                int np[3];
                int sign = 1;
                for (int r = 0; r < 3; ++r) {
                    np[p[r]] = n[r];
                    if (n[r] % 2 == 1) sign *= s[r];
                }
                G.src[g][k] = row_of_tensor(9 * np[2] + 3 * np[1] + np[0]);
                G.sign[g][k] = (float)sign;
            }
            ++g;
        }
    return G;
}

}  // namespace

struct nco_lattice {
    int nx = 0, ny = 0, nz = 0, n = 0;
    int storage = 0, op = 0;
    int domain = 0;               // DOMAIN_PERIODIC or DOMAIN_TGV_OCTANT
    double tau = 0.0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    size_t pop_bytes = 0;
    double omega_high[4] = {1.0, 1.0, 1.0, 1.0};
    float* net = nullptr;
    void* mfma_tab = nullptr;     // per-lane operand table + group gather table
    int width = 0, act = 0, mlp_prec = 0;
    int depth = 2;                // hidden layers
    int user_width = 0;           // width as given (a depth-3 network runs padded to 32)
    double* staging = nullptr;    // host-transfer staging, allocated on first use
    int staging_per_node = 0;     // its size in doubles per node
    double* partial = nullptr;    // global-sum partials
    double* small = nullptr;      // 64 doubles of results
    int* flag = nullptr;
    void* spec_work = nullptr;
    // Spectral forcing: coefficients of every step of the forcing period.
    int n_modes = 0, force_steps = 0;
    long force_t = 0;             // forcing step of the next lattice step
    int* d_fk = nullptr;
    double* d_fhat = nullptr;
    // The force synthesised on every node for the step about to run
    // ([3][n]; float64 for float64 storage, float32 otherwise) and the
    // largest |k_x| of the modes.
    void* d_force = nullptr;
    int force_kx = 0;
    // Velocity-dependent phase (Alvelius' rule): per-mode basis and |A|
    // [8 per mode], per-step draws phi, psi [steps][modes][2], mode-sum work
    // space and the coefficients of the current step.
    bool phase_rule = false;
    double* d_fbasis = nullptr;
    double* d_fdraw = nullptr;
    double* d_fpart = nullptr;
    double* d_fhat_cur = nullptr;
    // For the reverse mode: F_hat and u_hat of every recorded step
    // [steps][12 per mode] (capacity in doubles), and dL/du_hat [6 per mode].
    double* d_phist = nullptr;
    size_t phist_cap = 0;
    double* d_fduhat = nullptr;
    // Recorded forward run (checkpoints) for the adjoint.
    int rec_steps = -1, rec_every = 0;
    long rec_force_t0 = 0;
    long steps_since_record = 0;
    std::vector<void*> ckpt, seg;
    double* d_k = nullptr;        // energy samples of a recorded run (5 sums each)
    int d_k_cap = 0;
    float* lam[2] = {nullptr, nullptr};
    float* adj_partial = nullptr;
    size_t adj_partial_floats = 0;
    float* adj_xwork = nullptr;   // exchange space of the split depth-3 reverse step
    size_t adj_xwork_floats = 0;
    double* d_grad = nullptr;
    double* d_dE = nullptr;
    int* d_gsrc = nullptr;        // [48][27] group source row | sign bit
    // Matrix-core adjoint: float32 forward tables and the adjoint table
    // (width-32 networks on matrix cores), float64 per-block gradient rows.
    void* adj_tab = nullptr;
    double* adj_partial64 = nullptr;
    // Stability check: every check_every steps, the global sums are checked
    // on the device against the mass at the last initialisation; a failure
    // sets *flag, which nco_sync reports.
    int check_every = 0;
    double check_tol = 0.0;
    double mass0 = 0.0;
    long steps_since_check = 0;
    // Pairs of BGK / fixed-rate steps in place on one buffer when it fits
    // the last-level cache (nco_set_inplace; on by default).
    bool inplace = true;
    // Stochastic rounding of 16-bit deviation storage (nco_set_stochastic_rounding).
    bool sr = false;
    unsigned sr_seed = 0;
    // Reverse mode of float32 matrix-core networks: the network values each
    // recomputed forward step keeps for its adjoint (K - 1 states of a
    // segment), and those the recorded run kept for the last state of each
    // segment (net_ends, when rec_ends), within a budget of net_cache_bytes
    // (nco_set_reverse_cache).
    float* net_sums = nullptr;
    size_t net_sums_floats = 0;
    float* net_ends = nullptr;
    size_t net_ends_floats = 0;
    bool rec_ends = false;
    size_t net_cache_bytes = (size_t)4 << 30;
};

namespace {

int check_lat(nco_lattice* lat) {
    if (!lat) return fail(NCO_E_INVALID, "null lattice");
    return NCO_OK;
}

int set_device(nco_lattice* lat) {
    HIP_TRY(hipSetDevice(lat->device));
    return NCO_OK;
}

// Reference mass of the stability check (float64 sum of the state just set)
// and a cleared flag.  Synchronous.
int record_mass(nco_lattice* lat) {
    const int zero = 0;
    double sums[5];
    HIP_TRY(launch_global_sums(lat->storage, lat->f[lat->cur], lat->partial, lat->small, lat->n, lat->stream));
    HIP_TRY(hipMemcpyAsync(sums, lat->small, sizeof sums, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->flag, &zero, sizeof zero, hipMemcpyHostToDevice, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->mass0 = sums[0];
    lat->steps_since_check = 0;
    return NCO_OK;
}

// After a step queued on stream st: the stability check when it is due.
int maybe_check(nco_lattice* lat, hipStream_t st) {
    if (lat->check_every <= 0 || ++lat->steps_since_check < lat->check_every) return NCO_OK;
    lat->steps_since_check = 0;
    HIP_TRY(launch_check_state(lat->storage, lat->f[lat->cur], lat->partial, lat->small + 8, lat->n, lat->mass0,
                               lat->check_tol, lat->flag, st));
    return NCO_OK;
}

// Host-transfer staging of at least `per_node` doubles per node, grown on
// demand (4 for velocity and density fields, 27 for populations).
int ensure_staging(nco_lattice* lat, int per_node) {
    if (lat->staging_per_node >= per_node) return NCO_OK;
    if (lat->staging) {
        HIP_TRY(hipStreamSynchronize(lat->stream));
        HIP_TRY(hipFree(lat->staging));
        lat->staging = nullptr;
        lat->staging_per_node = 0;
    }
    HIP_TRY(hipMalloc(&lat->staging, sizeof(double) * per_node * (size_t)lat->n));
    lat->staging_per_node = per_node;
    return NCO_OK;
}

// Side streams and fork/join events of nco_batch_step, one set per device,
// created on first use (default priority) and kept until the process ends.
// g_side_mutex is held while a batch is enqueued, so that batches issued from
// several threads do not interleave their records of the shared events.
constexpr int BATCH_SIDE_STREAMS = 3;
constexpr int MAX_DEVICES = 64;
struct BatchSide {
    hipStream_t st[BATCH_SIDE_STREAMS] = {};
    hipEvent_t ev[1 + BATCH_SIDE_STREAMS] = {};
    bool ready = false;
};
BatchSide g_side[MAX_DEVICES];
std::mutex g_side_mutex;

int side_streams(int device, hipStream_t (&out)[BATCH_SIDE_STREAMS]) {
    if (device < 0 || device >= MAX_DEVICES) return fail(NCO_E_UNSUPPORTED, "device index %d", device);
    BatchSide& b = g_side[device];
    if (!b.ready) {
        for (int k = 0; k < BATCH_SIDE_STREAMS; ++k)
            HIP_TRY(hipStreamCreateWithFlags(&b.st[k], hipStreamNonBlocking));
        for (int k = 0; k < 1 + BATCH_SIDE_STREAMS; ++k)
            HIP_TRY(hipEventCreateWithFlags(&b.ev[k], hipEventDisableTiming));
        b.ready = true;
    }
    for (int k = 0; k < BATCH_SIDE_STREAMS; ++k) out[k] = b.st[k];
    return NCO_OK;
}

hipEvent_t batch_event(int device, int k) { return g_side[device].ev[k]; }

bool use_mfma(const nco_lattice* lat) {
    return lat->op == NCO_OP_NCO && lat->mlp_prec != NCO_MLP_F32 && lat->mfma_tab;
}
const float* mfma_lane_tab(const nco_lattice* lat) { return static_cast<const float*>(lat->mfma_tab); }
const int* mfma_group_tab(const nco_lattice* lat) {
    return reinterpret_cast<const int*>(static_cast<const char*>(lat->mfma_tab) +
                                        sizeof(float) * mfma_lane_table_floats());
}

StepArgs step_args(const nco_lattice* lat) {
    StepArgs a;
    a.nx = lat->nx;
    a.ny = lat->ny;
    a.nz = lat->nz;
    a.n = lat->n;
    a.op = lat->op;
    a.domain = lat->domain;
    a.width = lat->width;
    a.depth = lat->depth;
    a.act = lat->act;
    a.omega_nu = 1.0 / lat->tau;
    a.omega_nu_f = (float)a.omega_nu;
    for (int k = 0; k < 4; ++k) {
        a.omega_high[k] = lat->omega_high[k];
        a.omega_high_f[k] = (float)lat->omega_high[k];
    }
    a.net = lat->net;
    a.n_modes = 0;
    a.fk = nullptr;
    a.fhat = nullptr;
    a.force32 = nullptr;
    a.force64 = nullptr;
    a.sr_key = 0;
    a.net_sums = nullptr;
    return a;
}

// Arguments of the step that uses forcing step t.
StepArgs step_args_at(const nco_lattice* lat, long t) {
    StepArgs a = step_args(lat);
    // Each step's stochastic-rounding key from the lattice's seed and the
    // step index (never 0, which means round to nearest even).
    if (lat->sr) a.sr_key = lowbias32(lat->sr_seed ^ lowbias32((unsigned)t * 2654435769u)) | 1u;
    if (lat->n_modes > 0) {
        a.n_modes = lat->n_modes;
        a.fk = lat->d_fk;
        a.fhat = lat->d_fhat + (size_t)(t % lat->force_steps) * lat->n_modes * 6;
        if (lat->storage == NCO_F64)
            a.force64 = static_cast<const double*>(lat->d_force);
        else
            a.force32 = static_cast<const float*>(lat->d_force);
    }
    return a;
}

// The force field of the step with arguments a (a.fhat set), on stream st.
int force_field(nco_lattice* lat, const StepArgs& a, hipStream_t st) {
    if (a.n_modes <= 0) return NCO_OK;
    HIP_TRY(launch_force_field(a, lat->force_kx,
                               lat->storage == NCO_F64 ? nullptr : static_cast<float*>(lat->d_force),
                               lat->storage == NCO_F64 ? static_cast<double*>(lat->d_force) : nullptr, st));
    return NCO_OK;
}

// F_hat (then u_hat) of recorded step `slot` under the velocity-dependent phase.
double* phase_slot(const nco_lattice* lat, int slot) {
    return lat->d_phist + (size_t)slot * 12 * lat->n_modes;
}

// One forward step from buffer fin to fout with the given forcing step.
// Under the velocity-dependent phase, slot >= 0 keeps the step's F_hat and
// u_hat in recorded slot `slot`, and replay takes F_hat from that slot
// instead of computing it again.
// Two BGK or fixed-rate steps of nco_step run in place on one buffer when
// that buffer fits the last-level cache (256 MB on this device) and the pair
// of buffers does not: a 128^3 float32 lattice then stays cache-resident
// (measured 88.8 -> 71.5 us per step); larger lattices stream through HBM
// either way and keep the two-buffer step, whose non-temporal stores are
// faster there.  Periodic domain only, and not with the velocity-dependent
// forcing phase (it reads the state between the two steps).
constexpr size_t LLC_BYTES = (size_t)256 << 20;
bool inplace_pair_ok(const nco_lattice* lat) {
    return lat->inplace && (lat->op == NCO_OP_BGK || lat->op == NCO_OP_MRT) && lat->domain == NCO_DOMAIN_PERIODIC &&
           !lat->phase_rule && lat->pop_bytes <= LLC_BYTES && 2 * lat->pop_bytes > LLC_BYTES;
}

// Floats of the network values of one state (NET_SUMS_PER_NODE per node,
// the node count rounded up to whole 256-node blocks).
size_t net_values_stride(const nco_lattice* lat) { return (size_t)((lat->n + 255) / 256) * 256 * NET_SUMS_PER_NODE; }

// The reverse mode runs on the matrix cores and can read kept network values
// (float32 matrix-core network of depth 2).
bool net_values_apply(const nco_lattice* lat) {
    return lat->mlp_prec == NCO_MLP_F32_MFMA && lat->adj_tab && lat->depth == 2;
}

int launch_one(nco_lattice* lat, const void* fin, void* fout, long t, int slot = -1, bool replay = false,
               float* net_sums = nullptr) {
    StepArgs a = step_args_at(lat, t);
    a.net_sums = net_sums;
    if (lat->phase_rule && lat->n_modes > 0) {
        double* fh = slot >= 0 ? phase_slot(lat, slot) : lat->d_fhat_cur;
        // This step's coefficients from the velocity of the state it starts from.
        if (!replay)
            HIP_TRY(launch_force_phase(lat->storage, fin, lat->n, lat->nx, lat->ny, lat->nz, lat->d_fk,
                                       lat->n_modes, lat->d_fpart, lat->d_fbasis,
                                       lat->d_fdraw + (size_t)(t % lat->force_steps) * lat->n_modes * 2, fh,
                                       slot >= 0 ? fh + 6 * lat->n_modes : nullptr, lat->stream));
        a.fhat = fh;
    }
    if (int rc = force_field(lat, a, lat->stream)) return rc;
    if (use_mfma(lat))
        HIP_TRY(launch_nco_mfma(lat->storage, lat->mlp_prec, fin, fout, a, mfma_lane_tab(lat), mfma_group_tab(lat),
                                nullptr, lat->stream));
    else
        HIP_TRY(launch_step(lat->storage, fin, fout, a, lat->stream));
    return NCO_OK;
}

}  // namespace

extern "C" {

int nco_version(void) { return 100; }

const char* nco_last_error(void) { return g_err.c_str(); }

int nco_lattice_bytes(int nx, int ny, int nz, int storage, size_t* bytes) {
    if (nx < 1 || ny < 1 || nz < 1 || !bytes) return fail(NCO_E_INVALID, "bad size or null output");
    const size_t sb = store_bytes(storage);
    if (!sb) return fail(NCO_E_INVALID, "unknown storage %d", storage);
    const size_t n = (size_t)nx * ny * nz;
    // Two population buffers, the global-sum partials, the small result
    // area and the staging nco_init_equilibrium uses (4 doubles per node).
    *bytes = 2 * 27 * n * sb + 5 * sizeof(double) * ((n + 255) / 256) + 4096 + 4 * sizeof(double) * n;
    return NCO_OK;
}

int nco_lattice_create(int nx, int ny, int nz, int storage, int op, double tau, void* stream,
                       nco_lattice** out) {
    if (!out) return fail(NCO_E_INVALID, "null output pointer");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(NCO_E_INVALID, "lattice extent must be >= 1");
    const size_t n = (size_t)nx * ny * nz;
    if (n * 27 > (size_t)0x7fffffff * 8 || n > (size_t)0x7fffffff)
        return fail(NCO_E_INVALID, "lattice too large");
    if (!store_bytes(storage)) return fail(NCO_E_INVALID, "unknown storage %d", storage);
    if (op < NCO_OP_BGK || op > NCO_OP_STREAM) return fail(NCO_E_INVALID, "unknown operator %d", op);
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(NCO_E_INVALID, "tau must be > 1/2 (got %g)", tau);
    nco_lattice* lat = new nco_lattice;
    lat->nx = nx;
    lat->ny = ny;
    lat->nz = nz;
    lat->n = (int)n;
    lat->storage = storage;
    lat->op = op;
    lat->tau = tau;
    int rc = NCO_OK;
    auto bail = [&](int code) {
        nco_lattice_destroy(lat);
        return code;
    };
    if (hipGetDevice(&lat->device) != hipSuccess) return bail(fail(NCO_E_HIP, "hipGetDevice failed"));
    if (stream) {
        lat->stream = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&lat->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(NCO_E_HIP, "hipStreamCreate failed"));
        lat->own_stream = true;
    }
    lat->pop_bytes = 27 * n * store_bytes(storage);
    for (int b = 0; b < 2; ++b)
        if (hipMalloc(&lat->f[b], lat->pop_bytes) != hipSuccess)
            return bail(fail(NCO_E_OOM, "cannot allocate %zu bytes of populations", lat->pop_bytes));
    if (hipMalloc(&lat->partial, 5 * sizeof(double) * (size_t)sums_partial_count(lat->n)) != hipSuccess ||
        hipMalloc(&lat->small, 64 * sizeof(double)) != hipSuccess ||
        hipMalloc(&lat->flag, sizeof(int)) != hipSuccess)
        return bail(fail(NCO_E_OOM, "cannot allocate lattice work space"));
    // Rest state f = w (no host transfer, no staging).
    if (hipError_t e = launch_init_equilibrium(storage, lat->f[0], nullptr, nullptr, lat->n, lat->stream))
        return bail(fail(NCO_E_HIP, "rest state: %s", hipGetErrorString(e)));
    rc = record_mass(lat);
    if (rc != NCO_OK) return bail(rc);
    *out = lat;
    return NCO_OK;
}

int nco_lattice_destroy(nco_lattice* lat) {
    if (!lat) return NCO_OK;
    hipSetDevice(lat->device);
    if (lat->stream) hipStreamSynchronize(lat->stream);
    for (int b = 0; b < 2; ++b)
        if (lat->f[b]) hipFree(lat->f[b]);
    if (lat->net) hipFree(lat->net);
    if (lat->mfma_tab) hipFree(lat->mfma_tab);
    if (lat->staging) hipFree(lat->staging);
    if (lat->partial) hipFree(lat->partial);
    if (lat->small) hipFree(lat->small);
    if (lat->flag) hipFree(lat->flag);
    if (lat->adj_tab) hipFree(lat->adj_tab);
    if (lat->adj_partial64) hipFree(lat->adj_partial64);
    if (lat->net_sums) hipFree(lat->net_sums);
    if (lat->net_ends) hipFree(lat->net_ends);
    if (lat->spec_work) hipFree(lat->spec_work);
    if (lat->d_fk) hipFree(lat->d_fk);
    if (lat->d_fhat) hipFree(lat->d_fhat);
    if (lat->d_force) hipFree(lat->d_force);
    if (lat->d_fbasis) hipFree(lat->d_fbasis);
    if (lat->d_fdraw) hipFree(lat->d_fdraw);
    if (lat->d_fpart) hipFree(lat->d_fpart);
    if (lat->d_fhat_cur) hipFree(lat->d_fhat_cur);
    if (lat->d_phist) hipFree(lat->d_phist);
    if (lat->d_fduhat) hipFree(lat->d_fduhat);
    for (void* p : lat->ckpt) hipFree(p);
    for (void* p : lat->seg) hipFree(p);
    if (lat->d_k) hipFree(lat->d_k);
    for (int b = 0; b < 2; ++b)
        if (lat->lam[b]) hipFree(lat->lam[b]);
    if (lat->adj_partial) hipFree(lat->adj_partial);
    if (lat->adj_xwork) hipFree(lat->adj_xwork);
    if (lat->d_grad) hipFree(lat->d_grad);
    if (lat->d_dE) hipFree(lat->d_dE);
    if (lat->d_gsrc) hipFree(lat->d_gsrc);
    if (lat->own_stream && lat->stream) hipStreamDestroy(lat->stream);
    delete lat;
    return NCO_OK;
}

int nco_set_op(nco_lattice* lat, int op, double tau) {
    if (int rc = check_lat(lat)) return rc;
    if (op < NCO_OP_BGK || op > NCO_OP_STREAM) return fail(NCO_E_INVALID, "unknown operator %d", op);
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(NCO_E_INVALID, "tau must be > 1/2 (got %g)", tau);
    lat->op = op;
    lat->tau = tau;
    return NCO_OK;
}

int nco_set_domain(nco_lattice* lat, int domain) {
    if (int rc = check_lat(lat)) return rc;
    if (domain == NCO_DOMAIN_PERIODIC) {
        if (lat->domain != domain) lat->rec_steps = -1;
        lat->domain = domain;
        return NCO_OK;
    }
    if (domain != NCO_DOMAIN_TGV_OCTANT) return fail(NCO_E_INVALID, "unknown domain %d", domain);
    if (lat->nx != lat->ny || lat->nx != lat->nz) return fail(NCO_E_INVALID, "the reduced domain is a cube");
    if (lat->n_modes > 0) return fail(NCO_E_UNSUPPORTED, "spectral forcing needs the periodic domain");
    lat->domain = domain;
    lat->rec_steps = -1;  // a recorded run used the other streaming
    return NCO_OK;
}

int nco_set_rates(nco_lattice* lat, const double omega_high[4]) {
    if (int rc = check_lat(lat)) return rc;
    if (!omega_high) return fail(NCO_E_INVALID, "null rates");
    for (int k = 0; k < 4; ++k) {
        if (!(omega_high[k] > 0.0 && omega_high[k] < 2.0))
            return fail(NCO_E_INVALID, "rate omega_%d = %g outside (0, 2)", k + 3, omega_high[k]);
        lat->omega_high[k] = omega_high[k];
    }
    return NCO_OK;
}

int nco_set_net_weights(nco_lattice* lat, int width, int act, int mlp_prec, const float* params,
                        size_t n_params) {
    return nco_set_net_weights_depth(lat, 2, width, act, mlp_prec, params, n_params);
}

int nco_set_net_weights_depth(nco_lattice* lat, int depth, int width, int act, int mlp_prec, const float* params,
                              size_t n_params) {
    if (int rc = check_lat(lat)) return rc;
    if (depth != 2 && depth != 3) return fail(NCO_E_INVALID, "depth %d not supported (2, 3)", depth);
    if (!width_ok(width)) return fail(NCO_E_INVALID, "width %d not supported (8, 16, 20, 32)", width);
    if (act != NCO_ACT_TANH && act != NCO_ACT_RELU) return fail(NCO_E_INVALID, "unknown activation %d", act);
    if (mlp_prec != NCO_MLP_F32 && mlp_prec != NCO_MLP_F32_MFMA && mlp_prec != NCO_MLP_BF16 &&
        mlp_prec != NCO_MLP_F32_SPLIT)
        return fail(NCO_E_INVALID, "unknown network precision %d", mlp_prec);
    if (mlp_prec != NCO_MLP_F32 && lat->storage == NCO_F64)
        return fail(NCO_E_UNSUPPORTED, "the matrix-core network needs float32 or 16-bit storage");
    if (!params) return fail(NCO_E_INVALID, "null parameters");
    if (n_params != n_params_depth(width, depth))
        return fail(NCO_E_INVALID, "expected %zu parameters for width %d and depth %d, got %zu",
                    n_params_depth(width, depth), width, depth, n_params);
    // Depth 3 runs at width 32, narrower networks zero-padded.
    std::vector<float> padded3;
    if (depth == 3 && width < 32) {
        padded3 = pad_params(params, width, 3, 32);
        params = padded3.data();
    }
    const int W = depth == 3 ? 32 : width;
    static const GroupAction G = build_group_action();
    std::vector<float> buf(net_floats_depth(W, depth), 0.0f);
    const float* W1 = params;
    const float* b1 = W1 + 27 * W;
    const float* W2 = b1 + W;
    const float* b2 = W2 + W * W;
    const float* W2b = b2 + W;                      // depth 3 only
    const float* b2b = W2b + W * W;
    const float* W3 = depth == 3 ? b2b + W : b2 + W;
    const float* b3 = W3 + 4 * W;
    if (depth == 3) {
        std::memcpy(&buf[net_off_w2b(W)], W2b, sizeof(float) * W * W);
        std::memcpy(&buf[net_off_b2b(W)], b2b, sizeof(float) * W);
    }
    for (int g = 0; g < NGROUP; ++g)
        for (int k = 0; k < 27; ++k)
            for (int h = 0; h < W; ++h)
                buf[g * 27 * W + G.src[g][k] * W + h] = G.sign[g][k] * W1[k * W + h];
    std::memcpy(&buf[net_off_b1(W)], b1, sizeof(float) * W);
    std::memcpy(&buf[net_off_w2(W)], W2, sizeof(float) * W * W);
    std::memcpy(&buf[net_off_b2(W)], b2, sizeof(float) * W);
    std::memcpy(&buf[net_off_w3(W)], W3, sizeof(float) * W * 4);
    std::memcpy(&buf[net_off_b3(W)], b3, sizeof(float) * 4);
    if (int rc = set_device(lat)) return rc;
    if (lat->net && (lat->width != W || lat->depth != depth)) {
        HIP_TRY(hipStreamSynchronize(lat->stream));
        HIP_TRY(hipFree(lat->net));
        lat->net = nullptr;
    }
    if (!lat->net) HIP_TRY(hipMalloc(&lat->net, sizeof(float) * buf.size()));
    HIP_TRY(hipMemcpyAsync(lat->net, buf.data(), sizeof(float) * buf.size(), hipMemcpyHostToDevice,
                           lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->width = W;
    lat->user_width = width;
    lat->depth = depth;
    lat->act = act;
    lat->mlp_prec = mlp_prec;
    lat->rec_steps = -1;  // a recorded run used the previous network
    {
        // Group table of the adjoint: source row | sign bit per element and row.
        int gs[48 * 27];
        for (int g = 0; g < NGROUP; ++g)
            for (int k = 0; k < 27; ++k)
                gs[g * 27 + k] = G.src[g][k] | (G.sign[g][k] < 0.0f ? (int)0x80000000 : 0);
        if (!lat->d_gsrc) HIP_TRY(hipMalloc(&lat->d_gsrc, sizeof(gs)));
        HIP_TRY(hipMemcpyAsync(lat->d_gsrc, gs, sizeof(gs), hipMemcpyHostToDevice, lat->stream));
        HIP_TRY(hipStreamSynchronize(lat->stream));
    }
    if (mlp_prec != NCO_MLP_F32) {
        const size_t nf = mfma_lane_table_floats(), ni = mfma_group_table_ints();
        std::vector<char> tab(sizeof(float) * nf + sizeof(int) * ni);
        // Narrower networks run zero-padded to width 32: a padded hidden unit
        // has zero weights and bias and zero outgoing weights, so it adds
        // nothing to the next layer for either activation.
        std::vector<float> padded;
        const float* p32 = params;
        if (W < 32) {
            const int P = 32;
            padded.assign(n_params_for(P), 0.0f);
            float* q = padded.data();
            for (int k = 0; k < 27; ++k)
                for (int h = 0; h < W; ++h) q[k * P + h] = W1[k * W + h];
            q += 27 * P;
            for (int h = 0; h < W; ++h) q[h] = b1[h];
            q += P;
            for (int i = 0; i < W; ++i)
                for (int o = 0; o < W; ++o) q[i * P + o] = W2[i * W + o];
            q += P * P;
            for (int o = 0; o < W; ++o) q[o] = b2[o];
            q += P;
            for (int i = 0; i < W; ++i)
                for (int n = 0; n < 4; ++n) q[i * 4 + n] = W3[i * 4 + n];
            q += 4 * P;
            for (int n = 0; n < 4; ++n) q[n] = b3[n];
            p32 = padded.data();
        }
        mfma_prepare_tables(p32, act, mlp_prec, G.src, reinterpret_cast<float*>(tab.data()),
                            reinterpret_cast<int*>(tab.data() + sizeof(float) * nf), depth);
        if (!lat->mfma_tab) HIP_TRY(hipMalloc(&lat->mfma_tab, tab.size()));
        HIP_TRY(hipMemcpyAsync(lat->mfma_tab, tab.data(), tab.size(), hipMemcpyHostToDevice, lat->stream));
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (W == 32 && depth == 2) {
            // Reverse mode on the matrix cores: the float32 forward tables
            // (also for a bf16 network) and the adjoint's own table.
            const size_t na = mfma_adjoint_table_floats();
            std::vector<char> at(sizeof(float) * (nf + na) + sizeof(int) * ni);
            float* lt32 = reinterpret_cast<float*>(at.data());
            int* gt32 = reinterpret_cast<int*>(at.data() + sizeof(float) * nf);
            float* adj = reinterpret_cast<float*>(at.data() + sizeof(float) * nf + sizeof(int) * ni);
            mfma_prepare_tables(params, act, NCO_MLP_F32_MFMA, G.src, lt32, gt32);
            mfma_prepare_adjoint_table(params, adj);
            if (!lat->adj_tab) HIP_TRY(hipMalloc(&lat->adj_tab, at.size()));
            HIP_TRY(hipMemcpyAsync(lat->adj_tab, at.data(), at.size(), hipMemcpyHostToDevice, lat->stream));
            HIP_TRY(hipStreamSynchronize(lat->stream));
        }
    }
    return NCO_OK;
}

int nco_init_equilibrium(nco_lattice* lat, const double* rho, const double* u) {
    if (int rc = check_lat(lat)) return rc;
    if (!u) return fail(NCO_E_INVALID, "null velocity");
    if (int rc = set_device(lat)) return rc;
    if (int rc = ensure_staging(lat, 4)) return rc;
    const size_t n = lat->n;
    double* d_u = lat->staging;
    double* d_rho = rho ? lat->staging + 3 * n : nullptr;
    HIP_TRY(hipMemcpyAsync(d_u, u, sizeof(double) * 3 * n, hipMemcpyHostToDevice, lat->stream));
    if (rho) HIP_TRY(hipMemcpyAsync(d_rho, rho, sizeof(double) * n, hipMemcpyHostToDevice, lat->stream));
    HIP_TRY(launch_init_equilibrium(lat->storage, lat->f[lat->cur], d_rho, d_u, lat->n, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->rec_steps = -1;            // a recorded run no longer ends in this state
    return record_mass(lat);
}

int nco_restrict(const nco_lattice* fine, nco_lattice* coarse) {
    if (int rc = check_lat(coarse)) return rc;
    if (int rc = check_lat(const_cast<nco_lattice*>(fine))) return rc;
    if (fine == coarse) return fail(NCO_E_INVALID, "restriction needs two lattices");
    const int r = fine->nx / coarse->nx;
    if (r < 1 || fine->nx != r * coarse->nx || fine->ny != r * coarse->ny || fine->nz != r * coarse->nz)
        return fail(NCO_E_INVALID, "the fine extent must be the same integer multiple of the coarse one on every axis");
    if (fine->domain != NCO_DOMAIN_PERIODIC || coarse->domain != NCO_DOMAIN_PERIODIC)
        return fail(NCO_E_UNSUPPORTED, "restriction needs periodic lattices");
    if (fine->device != coarse->device) return fail(NCO_E_INVALID, "the lattices live on different devices");
    if (int rc = set_device(coarse)) return rc;
    HIP_TRY(hipStreamSynchronize(fine->stream));
    const double factor = r * coarse->tau / fine->tau;
    HIP_TRY(launch_restrict(fine->storage, fine->f[fine->cur], fine->nx, fine->ny, fine->nz, coarse->storage,
                            coarse->f[coarse->cur], coarse->nx, coarse->ny, coarse->nz, r, factor, coarse->stream));
    HIP_TRY(hipStreamSynchronize(coarse->stream));
    coarse->rec_steps = -1;
    return record_mass(coarse);
}

int nco_init_populations(nco_lattice* lat, const double* f) {
    if (int rc = check_lat(lat)) return rc;
    if (!f) return fail(NCO_E_INVALID, "null populations");
    if (int rc = set_device(lat)) return rc;
    if (int rc = ensure_staging(lat, 27)) return rc;
    HIP_TRY(hipMemcpyAsync(lat->staging, f, sizeof(double) * 27 * (size_t)lat->n, hipMemcpyHostToDevice,
                           lat->stream));
    HIP_TRY(launch_from_double(lat->storage, lat->f[lat->cur], lat->staging, lat->n, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->rec_steps = -1;
    return record_mass(lat);
}

int nco_step(nco_lattice* lat, int nsteps) {
    if (int rc = check_lat(lat)) return rc;
    if (nsteps < 0) return fail(NCO_E_INVALID, "nsteps must be >= 0");
    if (lat->op == NCO_OP_NCO && !lat->net) return fail(NCO_E_STATE, "NCO operator needs network weights");
    if (int rc = set_device(lat)) return rc;
    for (int s = 0; s < nsteps;) {
        // A pair in place never straddles a stability check: the state
        // between its two steps is in the swapped layout.
        const long to_check = lat->check_every > 0 ? lat->check_every - lat->steps_since_check : 2;
        if (nsteps - s >= 2 && to_check >= 2 && inplace_pair_ok(lat)) {
            for (int phase = 0; phase < 2; ++phase) {
                const StepArgs a = step_args_at(lat, lat->force_t);
                if (int rc = force_field(lat, a, lat->stream)) return rc;
                HIP_TRY(launch_step_inplace(lat->storage, lat->f[lat->cur], a, phase, lat->stream));
                ++lat->force_t;
                ++lat->steps_since_record;
                if (int rc = maybe_check(lat, lat->stream)) return rc;
            }
            s += 2;
            continue;
        }
        if (int rc = launch_one(lat, lat->f[lat->cur], lat->f[1 - lat->cur], lat->force_t)) return rc;
        lat->cur = 1 - lat->cur;
        ++lat->force_t;
        ++lat->steps_since_record;
        if (int rc = maybe_check(lat, lat->stream)) return rc;
        ++s;
    }
    return NCO_OK;
}

int nco_set_stochastic_rounding(nco_lattice* lat, int enable, unsigned seed) {
    if (int rc = check_lat(lat)) return rc;
    if (enable != 0 && enable != 1) return fail(NCO_E_INVALID, "enable must be 0 or 1");
    if (enable && lat->storage != NCO_BF16_DEV && lat->storage != NCO_F16_DEV)
        return fail(NCO_E_UNSUPPORTED, "stochastic rounding is for 16-bit deviation storage");
    lat->sr = enable == 1;
    lat->sr_seed = seed;
    lat->rec_steps = -1;  // a recorded run used the other rounding
    return NCO_OK;
}

int nco_set_reverse_cache(nco_lattice* lat, size_t bytes) {
    if (int rc = check_lat(lat)) return rc;
    lat->net_cache_bytes = bytes;
    return NCO_OK;
}

int nco_set_inplace(nco_lattice* lat, int enable) {
    if (int rc = check_lat(lat)) return rc;
    if (enable != 0 && enable != 1) return fail(NCO_E_INVALID, "enable must be 0 or 1");
    lat->inplace = enable == 1;
    return NCO_OK;
}

int nco_set_check(nco_lattice* lat, int every, double mass_rel_tol) {
    if (int rc = check_lat(lat)) return rc;
    if (every < 0 || !(mass_rel_tol >= 0.0)) return fail(NCO_E_INVALID, "every must be >= 0 and tolerance >= 0");
    if (int rc = set_device(lat)) return rc;
    lat->check_every = every;
    lat->check_tol = mass_rel_tol;
    return record_mass(lat);
}

int nco_batch_step(nco_lattice** lats, int n, const int* nsteps) {
    if (!lats || !nsteps || n < 0) return fail(NCO_E_INVALID, "null arguments");
    if (n == 0) return NCO_OK;
    nco_lattice* first = lats[0];
    int max_steps = 0;
    for (int i = 0; i < n; ++i) {
        nco_lattice* lat = lats[i];
        if (!lat) return fail(NCO_E_INVALID, "lattice %d is null", i);
        if (nsteps[i] < 0) return fail(NCO_E_INVALID, "nsteps[%d] < 0", i);
        if (lat->stream != first->stream || lat->device != first->device)
            return fail(NCO_E_INVALID, "all lattices of a batch must share one device and stream");
        for (int j = 0; j < i; ++j)
            if (lats[j] == lat) return fail(NCO_E_INVALID, "lattice %d appears twice", i);
        if (lat->op == NCO_OP_NCO && !use_mfma(lat))
            return fail(NCO_E_UNSUPPORTED, "batched NCO lattices need the matrix-core network (width 32)");
        if (lat->op == NCO_OP_STREAM) return fail(NCO_E_UNSUPPORTED, "batched streaming-only lattices");
        if (lat->phase_rule) return fail(NCO_E_UNSUPPORTED, "batched lattices with the velocity-dependent forcing phase");
        if (lat->depth != 2) return fail(NCO_E_UNSUPPORTED, "batched lattices with a third hidden layer");
        max_steps = std::max(max_steps, nsteps[i]);
    }
    if (int rc = set_device(first)) return rc;
    // Kernel kind of each lattice; chunks of up to GROUP_MAX lattices of one
    // kind share a dispatch per step.
    auto kind = [](const nco_lattice* l) {
        return l->op == NCO_OP_NCO ? 1000 + 100 * l->storage + 10 * l->mlp_prec + l->act : 10 * l->storage + l->op;
    };
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return kind(lats[x]) < kind(lats[y]); });
    std::vector<std::vector<int>> chunks;
    for (int pos = 0; pos < n;) {
        std::vector<int> c;
        const int k0 = kind(lats[order[pos]]);
        while (pos < n && kind(lats[order[pos]]) == k0 && (int)c.size() < GROUP_MAX) {
            if (nsteps[order[pos]] > 0) c.push_back(order[pos]);
            ++pos;
        }
        if (!c.empty()) chunks.push_back(std::move(c));
    }
    if (chunks.empty()) return NCO_OK;
    // Chunk 0 runs on the shared stream; the others on side streams forked
    // from it and joined back, so that chunks of different kinds (and the
    // chunks of a large batch) proceed concurrently.
    std::lock_guard<std::mutex> lock(g_side_mutex);
    hipStream_t side[BATCH_SIDE_STREAMS] = {};
    const int n_side = std::min((int)chunks.size() - 1, BATCH_SIDE_STREAMS);
    if (n_side > 0) {
        if (int rc = side_streams(first->device, side)) return rc;
        HIP_TRY(hipEventRecord(batch_event(first->device, 0), first->stream));
        for (int k = 0; k < n_side; ++k) HIP_TRY(hipStreamWaitEvent(side[k], batch_event(first->device, 0), 0));
    }
    for (size_t c = 0; c < chunks.size(); ++c) {
        hipStream_t st = c == 0 ? first->stream : side[(c - 1) % BATCH_SIDE_STREAMS];
        const std::vector<int>& mem = chunks[c];
        const nco_lattice* l0 = lats[mem[0]];
        int chunk_steps = 0;
        for (int idx : mem) chunk_steps = std::max(chunk_steps, nsteps[idx]);
        for (int s = 0; s < chunk_steps; ++s) {
            LaunchGroup g;
            g.count = 0;
            g.prefix[0] = 0;
            for (int idx : mem) {
                if (nsteps[idx] <= s) continue;
                nco_lattice* lat = lats[idx];
                GroupDesc& d = g.d[g.count];
                d.fin = lat->f[lat->cur];
                d.fout = lat->f[1 - lat->cur];
                d.a = step_args_at(lat, lat->force_t);
                if (int rc = force_field(lat, d.a, st)) return rc;
                d.lane_tab = lat->op == NCO_OP_NCO ? mfma_lane_tab(lat) : nullptr;
                d.gtab = lat->op == NCO_OP_NCO ? mfma_group_tab(lat) : nullptr;
                g.prefix[g.count + 1] = g.prefix[g.count] + (lat->n + 255) / 256;
                ++g.count;
                lat->cur = 1 - lat->cur;
                ++lat->force_t;
                ++lat->steps_since_record;
            }
            if (l0->op == NCO_OP_NCO)
                HIP_TRY(launch_nco_mfma_grouped(l0->storage, l0->mlp_prec, l0->act, g, st));
            else
                HIP_TRY(launch_step_grouped(l0->storage, l0->op, g, st));
            for (int idx : mem)
                if (nsteps[idx] > s)
                    if (int rc = maybe_check(lats[idx], st)) return rc;
        }
    }
    for (int k = 0; k < n_side; ++k) {
        HIP_TRY(hipEventRecord(batch_event(first->device, 1 + k), side[k]));
        HIP_TRY(hipStreamWaitEvent(first->stream, batch_event(first->device, 1 + k), 0));
    }
    return NCO_OK;
}

int nco_set_forcing(nco_lattice* lat, int n_modes, const int* k, const double* draws, int n_steps,
                    double amplitude, double kf, double c) {
    return nco_set_forcing_ex(lat, n_modes, k, draws, n_steps, amplitude, kf, c, 0);
}

int nco_set_forcing_ex(nco_lattice* lat, int n_modes, const int* k, const double* draws, int n_steps,
                       double amplitude, double kf, double c, int phase_rule) {
    if (int rc = check_lat(lat)) return rc;
    if (n_modes < 0 || (n_modes > 0 && (!k || !draws || n_steps < 1 || !(c > 0.0))))
        return fail(NCO_E_INVALID, "bad forcing arguments");
    if (phase_rule != 0 && phase_rule != 1) return fail(NCO_E_INVALID, "phase_rule must be 0 or 1");
    if (phase_rule && n_modes > 1024) return fail(NCO_E_INVALID, "at most 1024 modes with the phase rule");
    if (n_modes > 0 && lat->domain != NCO_DOMAIN_PERIODIC)
        return fail(NCO_E_UNSUPPORTED, "spectral forcing needs the periodic domain");
    int kx_max = 0;
    for (int m = 0; m < n_modes; ++m) kx_max = std::max(kx_max, std::abs(k[3 * m]));
    if (kx_max > FORCE_KX_MAX)
        return fail(NCO_E_UNSUPPORTED, "forced wavevectors need |k_x| <= %d (got %d)", FORCE_KX_MAX, kx_max);
    if (int rc = set_device(lat)) return rc;
    HIP_TRY(hipStreamSynchronize(lat->stream));
    if (lat->d_fk) HIP_TRY(hipFree(lat->d_fk));
    if (lat->d_fhat) HIP_TRY(hipFree(lat->d_fhat));
    if (lat->d_force) HIP_TRY(hipFree(lat->d_force));
    lat->d_fk = nullptr;
    lat->d_fhat = nullptr;
    lat->d_force = nullptr;
    lat->force_kx = 0;
    for (double** b : {&lat->d_fbasis, &lat->d_fdraw, &lat->d_fpart, &lat->d_fhat_cur, &lat->d_phist,
                       &lat->d_fduhat}) {
        if (*b) HIP_TRY(hipFree(*b));
        *b = nullptr;
    }
    lat->phist_cap = 0;
    lat->phase_rule = false;
    lat->rec_steps = -1;
    lat->n_modes = 0;
    lat->force_t = 0;
    if (n_modes == 0) return NCO_OK;
    // Alvelius coefficients (Sec. "Training Data - Forced Isotropic
    // Turbulence"): F_hat = A_ran e1 + B_ran e2 with A_ran, B_ran =
    // sqrt(F(k) / (2 pi k^2)) exp(i theta_{1,2}) (sin 2 phi, cos 2 phi),
    // theta2 = theta1 + psi, F(k) = amplitude exp(-(k - kf)^2 / c); e1 the
    // unit normal of k in the x-y plane, e2 = k x e1 / |k| as printed.
    std::vector<double> fh((size_t)n_steps * n_modes * 6);
    std::vector<double> basis((size_t)n_modes * 8, 0.0);
    for (int m = 0; m < n_modes; ++m) {
        const double kx = k[3 * m], ky = k[3 * m + 1], kz = k[3 * m + 2];
        const double kk = std::sqrt(kx * kx + ky * ky + kz * kz), kp = std::sqrt(kx * kx + ky * ky);
        if (!(kk > 0.0)) return fail(NCO_E_INVALID, "forcing wavevector %d is zero", m);
        double e1[3], e2[3];
        if (kp == 0.0) {
            e1[0] = 1; e1[1] = 0; e1[2] = 0;
            e2[0] = 0; e2[1] = 1; e2[2] = 0;
        } else {
            e1[0] = ky / kp; e1[1] = -kx / kp; e1[2] = 0.0;
            e2[0] = kx * kz / (kk * kp); e2[1] = ky * kz / (kk * kp); e2[2] = -kp / kk;
        }
        const double Fk = amplitude * std::exp(-(kk - kf) * (kk - kf) / c);
        const double mag = std::sqrt(Fk / (2.0 * M_PI * kk * kk));
        for (int a3 = 0; a3 < 3; ++a3) {
            basis[8 * m + a3] = e1[a3];
            basis[8 * m + 3 + a3] = e2[a3];
        }
        basis[8 * m + 6] = mag;
        for (int t = 0; t < n_steps; ++t) {
            const double* d = draws + ((size_t)t * n_modes + m) * 3;
            const double phi = M_PI * d[0], psi = 2.0 * M_PI * d[1], th1 = 2.0 * M_PI * d[2];
            const double ga = std::sin(2.0 * phi), gb = std::cos(2.0 * phi);
            const double Ar = mag * std::cos(th1) * ga, Ai = mag * std::sin(th1) * ga;
            const double Br = mag * std::cos(th1 + psi) * gb, Bi = mag * std::sin(th1 + psi) * gb;
            double* o = &fh[((size_t)t * n_modes + m) * 6];
            for (int a3 = 0; a3 < 3; ++a3) {
                o[2 * a3] = Ar * e1[a3] + Br * e2[a3];
                o[2 * a3 + 1] = Ai * e1[a3] + Bi * e2[a3];
            }
        }
    }
    HIP_TRY(hipMalloc(&lat->d_force, 3 * (size_t)lat->n * (lat->storage == NCO_F64 ? sizeof(double) : sizeof(float))));
    lat->force_kx = kx_max;
    HIP_TRY(hipMalloc(&lat->d_fk, sizeof(int) * 3 * n_modes));
    HIP_TRY(hipMalloc(&lat->d_fhat, sizeof(double) * fh.size()));
    HIP_TRY(hipMemcpyAsync(lat->d_fk, k, sizeof(int) * 3 * n_modes, hipMemcpyHostToDevice, lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->d_fhat, fh.data(), sizeof(double) * fh.size(), hipMemcpyHostToDevice, lat->stream));
    if (phase_rule) {
        // phi, psi of every step and mode (the theta1 draws are not used).
        std::vector<double> dr((size_t)n_steps * n_modes * 2);
        for (size_t e = 0; e < (size_t)n_steps * n_modes; ++e) {
            dr[2 * e] = M_PI * draws[3 * e];
            dr[2 * e + 1] = 2.0 * M_PI * draws[3 * e + 1];
        }
        HIP_TRY(hipMalloc(&lat->d_fbasis, sizeof(double) * basis.size()));
        HIP_TRY(hipMalloc(&lat->d_fdraw, sizeof(double) * dr.size()));
        HIP_TRY(hipMalloc(&lat->d_fpart, sizeof(double) * 6 * (size_t)n_modes * sums_partial_count(lat->n)));
        HIP_TRY(hipMalloc(&lat->d_fhat_cur, sizeof(double) * 6 * (size_t)n_modes));
        HIP_TRY(hipMalloc(&lat->d_fduhat, sizeof(double) * 6 * (size_t)n_modes));
        HIP_TRY(hipMemcpyAsync(lat->d_fbasis, basis.data(), sizeof(double) * basis.size(), hipMemcpyHostToDevice,
                               lat->stream));
        HIP_TRY(hipMemcpyAsync(lat->d_fdraw, dr.data(), sizeof(double) * dr.size(), hipMemcpyHostToDevice,
                               lat->stream));
        lat->phase_rule = true;
    }
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->n_modes = n_modes;
    lat->force_steps = n_steps;
    return NCO_OK;
}

int nco_forcing_amplitude(double power, double dt, double ka, double kb, double kf, double c,
                          double* amplitude) {
    if (!amplitude) return fail(NCO_E_INVALID, "null output");
    for (double v : {power, dt, ka, kb, kf, c})
        if (!std::isfinite(v)) return fail(NCO_E_INVALID, "non-finite forcing argument");
    if (power < 0.0 || !(dt > 0.0) || !(c > 0.0) || !(ka < kb))
        return fail(NCO_E_INVALID, "need power >= 0, dt > 0, c > 0 and ka < kb");
    // integral_{ka}^{kb} exp(-(k - kf)^2 / c) dk = sqrt(pi c) / 2 (erf(b) - erf(a))
    // with a, b the band edges in units of sqrt(c) from kf; the difference
    // of complementary error functions keeps its digits in the far tail.
    const double sc = std::sqrt(c), a = (ka - kf) / sc, b = (kb - kf) / sc;
    const double diff = a >= 0.0 ? std::erfc(a) - std::erfc(b) : b <= 0.0 ? std::erfc(-b) - std::erfc(-a)
                                                                       : std::erf(b) - std::erf(a);
    const double integral = 0.5 * std::sqrt(M_PI * c) * diff;
    if (!(integral > 0.0)) return fail(NCO_E_INVALID, "the forced band carries no weight (integral %g)", integral);
    *amplitude = (power / dt) / integral;
    return NCO_OK;
}

int nco_set_forcing_power(nco_lattice* lat, int n_modes, const int* k, const double* draws, int n_steps,
                          double power, double ka, double kb, double kf, double c, int phase_rule) {
    if (int rc = check_lat(lat)) return rc;
    double amplitude = 0.0;
    if (n_modes > 0)
        if (int rc = nco_forcing_amplitude(power, 1.0, ka, kb, kf, c, &amplitude)) return rc;
    return nco_set_forcing_ex(lat, n_modes, k, draws, n_steps, amplitude, kf, c, phase_rule);
}

namespace {

// Recorded forward run; every > 0: k(t) = <|u|^2> / 2 at t = 0, every, ...
// into k (host, nsteps / every + 1 values).
int forward_record(nco_lattice* lat, int nsteps, int ckpt_every, int every, double* k) {
    if (int rc = check_lat(lat)) return rc;
    if (nsteps < 1 || ckpt_every < 1) return fail(NCO_E_INVALID, "nsteps and ckpt_every must be >= 1");
    if (every < 0 || (every > 0 && !k)) return fail(NCO_E_INVALID, "energy sampling needs every >= 1 and an output");
    if (lat->op != NCO_OP_NCO || !lat->net) return fail(NCO_E_STATE, "recording needs the NCO operator with weights");
    if (lat->width != 32 || lat->storage == NCO_F64)
        return fail(NCO_E_UNSUPPORTED, "the adjoint needs width 32 and float storage");
    if (int rc = set_device(lat)) return rc;
    if (lat->phase_rule && lat->n_modes > 0) {
        const size_t need = (size_t)nsteps * 12 * lat->n_modes;
        if (need > lat->phist_cap) {
            HIP_TRY(hipStreamSynchronize(lat->stream));
            if (lat->d_phist) HIP_TRY(hipFree(lat->d_phist));
            lat->d_phist = nullptr;
            lat->phist_cap = 0;
            HIP_TRY(hipMalloc(&lat->d_phist, sizeof(double) * need));
            lat->phist_cap = need;
        }
    }
    const int ncp = (nsteps + ckpt_every - 1) / ckpt_every;
    while ((int)lat->ckpt.size() < ncp) {
        void* p = nullptr;
        HIP_TRY(hipMalloc(&p, lat->pop_bytes));
        lat->ckpt.push_back(p);
    }
    // The last step of each segment keeps its network values for the adjoint
    // of its state (no recomputed step precedes that adjoint) when they fit
    // the budget beside the recompute's K - 1 states.
    const size_t stride = net_values_stride(lat);
    const size_t ends_floats = (size_t)ncp * stride;
    lat->rec_ends = net_values_apply(lat) &&
                    ((size_t)(ckpt_every - 1) * stride + ends_floats) * sizeof(float) <= lat->net_cache_bytes;
    if (lat->rec_ends && lat->net_ends_floats < ends_floats) {
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (lat->net_ends) HIP_TRY(hipFree(lat->net_ends));
        lat->net_ends = nullptr;
        lat->net_ends_floats = 0;
        HIP_TRY(hipMalloc(&lat->net_ends, sizeof(float) * ends_floats));
        lat->net_ends_floats = ends_floats;
    }
    const int nk = every > 0 ? nsteps / every + 1 : 0;
    if (nk > lat->d_k_cap) {
        // Kept between calls: a free would wait for the whole device.
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (lat->d_k) HIP_TRY(hipFree(lat->d_k));
        lat->d_k = nullptr;
        lat->d_k_cap = 0;
        HIP_TRY(hipMalloc(&lat->d_k, sizeof(double) * 5 * nk));
        lat->d_k_cap = nk;
    }
    double* d_k = lat->d_k;
    auto sample = [&](int m) -> int {
        HIP_TRY(launch_global_sums(lat->storage, lat->f[lat->cur], lat->partial, d_k + 5 * m, lat->n, lat->stream));
        return NCO_OK;
    };
    int rc = NCO_OK;
    lat->rec_force_t0 = lat->force_t;
    if (nk > 0) rc = sample(0);
    for (int s = 0; s < nsteps && rc == NCO_OK; ++s) {
        if (s % ckpt_every == 0) {
            // The checkpoint takes over the buffer that holds the state (no
            // copy; every buffer has the lattice's size), the step reads it
            // there, and the checkpoint's previous buffer joins the two step
            // buffers (nco_device_populations' pointer is valid until the
            // next step).
            std::swap(lat->ckpt[s / ckpt_every], lat->f[lat->cur]);
        }
        const void* fin = s % ckpt_every == 0 ? lat->ckpt[s / ckpt_every] : lat->f[lat->cur];
        float* ends = lat->rec_ends && (s % ckpt_every == ckpt_every - 1 || s == nsteps - 1)
                          ? lat->net_ends + (size_t)(s / ckpt_every) * stride
                          : nullptr;
        if ((rc = launch_one(lat, fin, lat->f[1 - lat->cur], lat->force_t, s, false, ends))) break;
        lat->cur = 1 - lat->cur;
        ++lat->force_t;
        if (nk > 0 && (s + 1) % every == 0) rc = sample((s + 1) / every);
    }
    if (rc == NCO_OK && nk > 0) {
        std::vector<double> sums(5 * (size_t)nk);
        if (hipMemcpyAsync(sums.data(), d_k, sizeof(double) * sums.size(), hipMemcpyDeviceToHost, lat->stream) !=
                hipSuccess ||
            hipStreamSynchronize(lat->stream) != hipSuccess)
            rc = fail(NCO_E_HIP, "reading the energy samples failed");
        for (int m = 0; m < nk && rc == NCO_OK; ++m) k[m] = sums[5 * m + 4] / lat->n;
    }
    if (rc != NCO_OK) return rc;
    lat->rec_steps = nsteps;
    lat->rec_every = ckpt_every;
    lat->steps_since_record = 0;
    return NCO_OK;
}

}  // namespace

int nco_forward_record(nco_lattice* lat, int nsteps, int ckpt_every) {
    return forward_record(lat, nsteps, ckpt_every, 0, nullptr);
}

int nco_forward_record_energy(nco_lattice* lat, int nsteps, int ckpt_every, int every, double* k) {
    return forward_record(lat, nsteps, ckpt_every, every, k);
}

namespace {

int backward(nco_lattice* lat, const double* dL_dk, int every, const double* dL_dE, int nbins, const double* dL_df,
             double* grad, size_t n_params, double* dL_df0) {
    if (int rc = check_lat(lat)) return rc;
    if (lat->rec_steps < 1 || lat->steps_since_record != 0)
        return fail(NCO_E_STATE, "backward needs nco_forward_record immediately before it");
    const size_t want = lat->depth == 3 ? n_params_depth(lat->user_width, 3) : (size_t)adjoint_param_count();
    if (!grad || n_params != want) return fail(NCO_E_INVALID, "grad must hold %zu values", want);
    if (!dL_dE && !dL_df && !dL_dk) return fail(NCO_E_INVALID, "give dL_dE, dL_df or dL_dk");
    if (dL_dE && lat->domain != NCO_DOMAIN_PERIODIC)
        return fail(NCO_E_UNSUPPORTED, "a spectrum loss needs the periodic domain");
    if (dL_dk && every < 1) return fail(NCO_E_INVALID, "energy sampling needs every >= 1");
    // dL/dk(t) enters the adjoint of the state after t steps, t = m every.
    auto inject = [&](int t, const void* state, float* lam) -> int {
        if (!dL_dk || t % every != 0) return NCO_OK;
        const double g = dL_dk[t / every];
        if (g != 0.0) HIP_TRY(launch_add_energy_grad(lat->storage, state, lam, g / lat->n, lat->n, lat->stream));
        return NCO_OK;
    };
    if (int rc = set_device(lat)) return rc;
    const size_t n = lat->n, nf = 27 * n;
    if (dL_dE) {
        if (lat->nx != lat->ny || lat->nx != lat->nz) return fail(NCO_E_INVALID, "spectrum needs a cubic lattice");
        if (nbins != spectrum_bins(lat->nx)) return fail(NCO_E_INVALID, "nbins must be %d", spectrum_bins(lat->nx));
    }
    for (int b = 0; b < 2; ++b)
        if (!lat->lam[b]) HIP_TRY(hipMalloc(&lat->lam[b], sizeof(float) * nf));
    // Matrix-core adjoint for matrix-core networks, vector-unit adjoint for
    // the vector-unit network.
    // (a depth-3 network takes the vector-unit adjoint)
    const bool mfma = lat->mlp_prec != NCO_MLP_F32 && lat->adj_tab && lat->depth == 2;
    const int npar = mfma ? adjoint_param_count() : adjoint_param_count_depth(lat->depth);
    const int nblk = mfma ? adjoint_mfma_blocks(lat->n) : adjoint_blocks(lat->n, lat->depth);
    const int ngrp = (nblk + 63) / 64;
    if (mfma) {
        if (!lat->adj_partial64)
            HIP_TRY(hipMalloc(&lat->adj_partial64, sizeof(double) * (size_t)(nblk + ngrp) * npar));
        HIP_TRY(launch_fill_f64(lat->adj_partial64, (size_t)nblk * npar, 0.0, lat->stream));
    } else if (lat->adj_partial_floats < (size_t)nblk * npar) {
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (lat->adj_partial) HIP_TRY(hipFree(lat->adj_partial));
        lat->adj_partial = nullptr;
        lat->adj_partial_floats = 0;
        HIP_TRY(hipMalloc(&lat->adj_partial, sizeof(float) * (size_t)nblk * npar));
        lat->adj_partial_floats = (size_t)nblk * npar;
    }
    if (!mfma && adjoint_xwork_floats(lat->n, lat->depth) > lat->adj_xwork_floats) {
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (lat->adj_xwork) HIP_TRY(hipFree(lat->adj_xwork));
        lat->adj_xwork = nullptr;
        lat->adj_xwork_floats = 0;
        const size_t nx = adjoint_xwork_floats(lat->n, lat->depth);
        HIP_TRY(hipMalloc(&lat->adj_xwork, sizeof(float) * nx));
        lat->adj_xwork_floats = nx;
    }
    if (!lat->d_grad) HIP_TRY(hipMalloc(&lat->d_grad, sizeof(double) * adjoint_param_count_depth(3)));
    // Float32 matrix-core networks: each recomputed forward step keeps its
    // network values (group sums and tilde tau), and the adjoint of that
    // step reads them instead of running the network forward again (the
    // same arithmetic on the same state: the gradient is unchanged, bit for
    // bit).  The last state of a segment has no recomputed step and runs it.
    // The last state of a segment reads what the recorded run kept for it
    // (rec_ends), if it did.
    const size_t sums_stride = net_values_stride(lat);
    const bool keep_sums = mfma && net_values_apply(lat) && lat->rec_every > 1 &&
                           (size_t)(lat->rec_every - 1) * sums_stride * sizeof(float) <= lat->net_cache_bytes;
    if (keep_sums && lat->net_sums_floats < (size_t)(lat->rec_every - 1) * sums_stride) {
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (lat->net_sums) HIP_TRY(hipFree(lat->net_sums));
        lat->net_sums = nullptr;
        lat->net_sums_floats = 0;
        HIP_TRY(hipMalloc(&lat->net_sums, sizeof(float) * (size_t)(lat->rec_every - 1) * sums_stride));
        lat->net_sums_floats = (size_t)(lat->rec_every - 1) * sums_stride;
    }
    auto sums_of = [&](int i) { return keep_sums ? lat->net_sums + (size_t)i * sums_stride : nullptr; };
    auto end_of = [&](int sgi) { return lat->rec_ends ? lat->net_ends + (size_t)sgi * sums_stride : nullptr; };
    // States 1..K-1 of a segment (its state 0 is the checkpoint).
    while ((int)lat->seg.size() < lat->rec_every) {
        void* p = nullptr;
        if (!lat->seg.empty()) HIP_TRY(hipMalloc(&p, lat->pop_bytes));
        lat->seg.push_back(p);
    }
    // Adjoint of the final state.
    float* lin = lat->lam[0];
    float* lout = lat->lam[1];
    HIP_TRY(launch_fill_f32(lin, nf, 0.0f, lat->stream));
    if (dL_dE) {
        const int nn = lat->nx;
        if (!lat->spec_work) HIP_TRY(hipMalloc(&lat->spec_work, spectrum_workspace_bytes(nn) + 256 * sizeof(double) * 8));
        if (!lat->d_dE) HIP_TRY(hipMalloc(&lat->d_dE, sizeof(double) * 2048));
        if (nbins > 2048) return fail(NCO_E_UNSUPPORTED, "too many shells");
        HIP_TRY(hipMemcpyAsync(lat->d_dE, dL_dE, sizeof(double) * nbins, hipMemcpyHostToDevice, lat->stream));
        HIP_TRY(launch_spectrum_adjoint(lat->storage, lat->f[lat->cur], nn, lat->spec_work, lat->d_dE, nbins, lin,
                                        lat->stream));
    }
    if (dL_df) {
        if (int rc = ensure_staging(lat, 27)) return rc;
        HIP_TRY(hipMemcpyAsync(lat->staging, dL_df, sizeof(double) * nf, hipMemcpyHostToDevice, lat->stream));
        HIP_TRY(launch_add_f64_to_f32(lin, lat->staging, nf, lat->stream));
    }
    if (int rc = inject(lat->rec_steps, lat->f[lat->cur], lin)) return rc;
    HIP_TRY(launch_fill_f64(lat->d_grad, npar, 0.0, lat->stream));
    const int T = lat->rec_steps, K = lat->rec_every;
    const int ncp = (T + K - 1) / K;
    for (int sgi = ncp - 1; sgi >= 0; --sgi) {
        const int t0 = sgi * K, len = std::min(K, T - t0);
        // Recompute the states of this segment from its checkpoint, which
        // serves as the segment's first state itself (only read from here).
        auto state = [&](int i) -> void* { return i == 0 ? lat->ckpt[sgi] : lat->seg[i]; };
        for (int i = 1; i < len; ++i)
            if (int rc = launch_one(lat, state(i - 1), lat->seg[i], lat->rec_force_t0 + t0 + i - 1, t0 + i - 1,
                                    true, sums_of(i - 1)))
                return rc;
        for (int t = t0 + len - 1; t >= t0; --t) {
            StepArgs a = step_args_at(lat, lat->rec_force_t0 + t);
            const bool phase = lat->phase_rule && lat->n_modes > 0;
            if (phase) a.fhat = phase_slot(lat, t);
            if (int rc = force_field(lat, a, lat->stream)) return rc;
            if (mfma) {
                a.net_sums = t - t0 < len - 1 ? sums_of(t - t0) : end_of(sgi);
                const char* tab = static_cast<const char*>(lat->adj_tab);
                const float* lt32 = reinterpret_cast<const float*>(tab);
                const int* gt32 = reinterpret_cast<const int*>(tab + sizeof(float) * mfma_lane_table_floats());
                const float* adj = reinterpret_cast<const float*>(tab + sizeof(float) * mfma_lane_table_floats() +
                                                                  sizeof(int) * mfma_group_table_ints());
                HIP_TRY(launch_adjoint_mfma(lat->storage, lat->act, state(t - t0), lin, lout, a, lt32, gt32, adj,
                                            lat->d_gsrc, lat->adj_partial64, lat->stream));
            } else {
                HIP_TRY(launch_adjoint(lat->storage, state(t - t0), lin, lout, a, lat->d_gsrc, lat->adj_partial,
                                       lat->adj_xwork, lat->stream));
                HIP_TRY(launch_grad_reduce(lat->adj_partial, nblk, npar, lat->d_grad, lat->stream));
            }
            if (phase) {
                // The force of step t also depends on x_t through its velocity modes.
                const long ft = (lat->rec_force_t0 + t) % lat->force_steps;
                HIP_TRY(launch_force_phase_adjoint(lat->storage, state(t - t0), lin, lout, a, lat->d_fpart,
                                                   lat->d_fbasis, lat->d_fdraw + (size_t)ft * lat->n_modes * 2,
                                                   phase_slot(lat, t) + 6 * lat->n_modes, lat->d_fduhat,
                                                   lat->stream));
            }
            if (int rc = inject(t, state(t - t0), lout)) return rc;
            std::swap(lin, lout);
        }
    }
    if (mfma)
        HIP_TRY(launch_grad_reduce_f64(lat->adj_partial64, nblk, lat->adj_partial64 + (size_t)nblk * npar,
                                       lat->d_grad, lat->stream));
    if (dL_df0) {
        if (int rc = ensure_staging(lat, 27)) return rc;
        HIP_TRY(launch_f32_to_f64(lin, lat->staging, nf, lat->stream));
        HIP_TRY(hipMemcpyAsync(dL_df0, lat->staging, sizeof(double) * nf, hipMemcpyDeviceToHost, lat->stream));
    }
    // Last before the wait, so that no early return leaves a copy into g3 in flight.
    std::vector<double> g3(lat->depth == 3 ? npar : 0);
    HIP_TRY(hipMemcpyAsync(lat->depth == 3 ? g3.data() : grad, lat->d_grad, sizeof(double) * npar,
                           hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    if (lat->depth == 3) unpad_grad3(g3.data(), lat->width, lat->user_width, grad);
    return NCO_OK;
}

}  // namespace

int nco_backward(nco_lattice* lat, const double* dL_dE, int nbins, const double* dL_df, double* grad,
                 size_t n_params, double* dL_df0) {
    return backward(lat, nullptr, 0, dL_dE, nbins, dL_df, grad, n_params, dL_df0);
}

int nco_backward_energy(nco_lattice* lat, const double* dL_dk, int every, const double* dL_dE, int nbins,
                        const double* dL_df, double* grad, size_t n_params, double* dL_df0) {
    if (!dL_dk) return fail(NCO_E_INVALID, "null dL_dk");
    return backward(lat, dL_dk, every, dL_dE, nbins, dL_df, grad, n_params, dL_df0);
}

int nco_sync(nco_lattice* lat) {
    if (int rc = check_lat(lat)) return rc;
    if (int rc = set_device(lat)) return rc;
    HIP_TRY(hipStreamSynchronize(lat->stream));
    if (lat->check_every > 0) {
        int flag = 0;
        HIP_TRY(hipMemcpyAsync(&flag, lat->flag, sizeof flag, hipMemcpyDeviceToHost, lat->stream));
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (flag)
            return fail(NCO_E_UNSTABLE, "stability check failed: non-finite state or mass drift above %g",
                        lat->check_tol);
    }
    return NCO_OK;
}

int nco_read_populations(nco_lattice* lat, double* f) {
    if (int rc = check_lat(lat)) return rc;
    if (!f) return fail(NCO_E_INVALID, "null output");
    if (int rc = set_device(lat)) return rc;
    if (int rc = ensure_staging(lat, 27)) return rc;
    HIP_TRY(launch_to_double(lat->storage, lat->f[lat->cur], lat->staging, lat->n, lat->stream));
    HIP_TRY(hipMemcpyAsync(f, lat->staging, sizeof(double) * 27 * (size_t)lat->n, hipMemcpyDeviceToHost,
                           lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return NCO_OK;
}

int nco_read_macroscopic(nco_lattice* lat, double* rho, double* u) {
    if (int rc = check_lat(lat)) return rc;
    if (int rc = set_device(lat)) return rc;
    if (int rc = ensure_staging(lat, 4)) return rc;
    const size_t n = lat->n;
    HIP_TRY(launch_macroscopic(lat->storage, lat->f[lat->cur], lat->staging, lat->staging + n, lat->n,
                               lat->stream));
    if (rho) HIP_TRY(hipMemcpyAsync(rho, lat->staging, sizeof(double) * n, hipMemcpyDeviceToHost, lat->stream));
    if (u) HIP_TRY(hipMemcpyAsync(u, lat->staging + n, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return NCO_OK;
}

int nco_read_rates(nco_lattice* lat, double* omega) {
    if (int rc = check_lat(lat)) return rc;
    if (!omega) return fail(NCO_E_INVALID, "null output");
    if (!lat->net) return fail(NCO_E_STATE, "no network weights set");
    if (int rc = set_device(lat)) return rc;
    if (int rc = ensure_staging(lat, 4)) return rc;
    const StepArgs a = step_args(lat);
    if (use_mfma(lat))
        HIP_TRY(launch_nco_mfma(lat->storage, lat->mlp_prec, lat->f[lat->cur], nullptr, a, mfma_lane_tab(lat),
                                mfma_group_tab(lat), lat->staging, lat->stream));
    else
        HIP_TRY(launch_rates(lat->storage, lat->f[lat->cur], lat->staging, a, lat->stream));
    HIP_TRY(hipMemcpyAsync(omega, lat->staging, sizeof(double) * 4 * (size_t)lat->n, hipMemcpyDeviceToHost,
                           lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return NCO_OK;
}

int nco_global_sums(nco_lattice* lat, double out[5]) {
    if (int rc = check_lat(lat)) return rc;
    if (!out) return fail(NCO_E_INVALID, "null output");
    if (int rc = set_device(lat)) return rc;
    HIP_TRY(launch_global_sums(lat->storage, lat->f[lat->cur], lat->partial, lat->small, lat->n, lat->stream));
    HIP_TRY(hipMemcpyAsync(out, lat->small, 5 * sizeof(double), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(out[k])) return fail(NCO_E_UNSTABLE, "non-finite global sum %d", k);
    return NCO_OK;
}

int nco_energy_spectrum(nco_lattice* lat, double* E, int nbins) {
    if (int rc = check_lat(lat)) return rc;
    if (!E) return fail(NCO_E_INVALID, "null output");
    if (lat->nx != lat->ny || lat->nx != lat->nz) return fail(NCO_E_INVALID, "spectrum needs a cubic lattice");
    if (lat->domain != NCO_DOMAIN_PERIODIC) return fail(NCO_E_UNSUPPORTED, "spectrum needs the periodic domain");
    const int n = lat->nx;
    if (nbins != spectrum_bins(n)) return fail(NCO_E_INVALID, "nbins must be %d for n = %d", spectrum_bins(n), n);
    if (int rc = set_device(lat)) return rc;
    if (!lat->spec_work) HIP_TRY(hipMalloc(&lat->spec_work, spectrum_workspace_bytes(n) + 256 * sizeof(double) * 8));
    double* E_dev = reinterpret_cast<double*>(static_cast<char*>(lat->spec_work) + spectrum_workspace_bytes(n));
    if (nbins > 256 * 8) return fail(NCO_E_UNSUPPORTED, "too many shells");
    HIP_TRY(launch_energy_spectrum(lat->storage, lat->f[lat->cur], n, lat->spec_work, E_dev, nbins, lat->stream));
    HIP_TRY(hipMemcpyAsync(E, E_dev, sizeof(double) * nbins, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return NCO_OK;
}

int nco_energy_spectrum_noalloc(nco_lattice* lat, double* E_dev, int nbins) {
    if (int rc = check_lat(lat)) return rc;
    if (!E_dev) return fail(NCO_E_INVALID, "null output");
    if (lat->nx != lat->ny || lat->nx != lat->nz) return fail(NCO_E_INVALID, "spectrum needs a cubic lattice");
    if (lat->domain != NCO_DOMAIN_PERIODIC) return fail(NCO_E_UNSUPPORTED, "spectrum needs the periodic domain");
    const int n = lat->nx;
    if (nbins != spectrum_bins(n)) return fail(NCO_E_INVALID, "nbins must be %d for n = %d", spectrum_bins(n), n);
    const size_t need = spectrum_forward_bytes(n);
    if (need > spectrum_scratch_bytes())
        return fail(NCO_E_INVALID, "a %d^3 spectrum needs %zu bytes of scratch; the allocation-free spectrum has %zu",
                    n, need, spectrum_scratch_bytes());
    if (int rc = set_device(lat)) return rc;
    void* work = nullptr;
    HIP_TRY(spectrum_scratch(lat->device, &work));
    HIP_TRY(launch_energy_spectrum(lat->storage, lat->f[lat->cur], n, work, E_dev, nbins, lat->stream));
    return NCO_OK;
}

int nco_device_populations(nco_lattice* lat, void** dev_ptr, size_t* bytes) {
    if (int rc = check_lat(lat)) return rc;
    if (!dev_ptr || !bytes) return fail(NCO_E_INVALID, "null output");
    *dev_ptr = lat->f[lat->cur];
    *bytes = lat->pop_bytes;
    return NCO_OK;
}

}  // extern "C"
