// Host side of liblbm.so: workspace planning, tape (checkpoint + segment
// recompute) scheduling, parameter upload and the C ABI declared in lbm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_kernels.hpp"
#include "lbm_error.hpp"

using lbm::InstDev;

namespace {
thread_local std::string g_err;
}

// Records the detail of a failure for lbm_last_error() and returns code.
int lbm_fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace {

#define fail lbm_fail

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(LBM_EDEVICE, "%s failed: %s (%d)", #expr, hipGetErrorString(e_), (int)e_); \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device workspace layout of one problem.
struct Layout {
    int q = 9, D = 2, n_inst = 0;
    int T = 1, K = 1, n_seg = 1, tape = 0;
    int R = 1;                // resident segments: the last R segments' states are kept by the forward
    int frames = 1, stride = 1;   // loss frames: the states after steps T - (frames - 1 - m) stride
    int n_tiles = 0, n_ftiles = 0;
    long long total_poff = 0, total_nodes = 0, total_face = 0, total_words = 0;
    long long S = 0;          // floats per state buffer
    int n_states = 0;
    size_t off_inst = 0, off_mask = 0, off_roi = 0, off_target = 0, off_face_in = 0, off_face_out = 0,
           off_grad_in = 0, off_grad_out = 0, off_part_loss = 0, off_part_dtau = 0, off_part_res = 0,
           off_red = 0, off_fblk = 0, off_u2 = 0, off_seed = 0, off_flag = 0, off_states = 0, state_bytes = 0,
           total = 0;
    std::vector<InstDev> inst;
};

long long count_fluid(const lbm_instance &S);

// The kernels address one instance's populations through a buffer resource
// whose byte range and offsets are 32-bit: Q planes of the fluid nodes
// (padded to 64) must stay below 4 GiB.
constexpr long long MAX_INSTANCE_STATE_BYTES = (1LL << 32) - 1;

int validate_problem(const lbm_problem *p) {
    if (!p) return fail(LBM_EINVAL, "problem is NULL");
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19)
        return fail(LBM_EINVAL, "lattice must be LBM_D2Q9 or LBM_D3Q19 (got %d)", p->lattice);
    if (p->n_inst < 1 || !p->inst) return fail(LBM_EINVAL, "n_inst must be >= 1 with a descriptor array");
    if (p->resident_segments < 0)
        return fail(LBM_EINVAL, "resident_segments must be >= 0 (got %d)", p->resident_segments);
    if (p->loss_frames < 0) return fail(LBM_EINVAL, "loss_frames must be >= 0 (got %d)", p->loss_frames);
    if (p->loss_frames > 1 && (p->loss_stride < 1 || (long long)(p->loss_frames - 1) * p->loss_stride >= p->steps))
        return fail(LBM_EINVAL, "loss frames must lie on steps 1 .. T: need loss_stride >= 1 and "
                                "(loss_frames - 1) loss_stride < T (got %d frames, stride %d, T %d)",
                    p->loss_frames, p->loss_stride, p->steps);
    const int bcs[3] = {p->bc_x, p->bc_y, p->bc_z};
    for (int a = 0; a < 3; ++a)
        if (bcs[a] < LBM_BC_PRESSURE || bcs[a] > LBM_BC_VELOCITY)
            return fail(LBM_EINVAL, "boundary kind of axis %d is invalid (%d)", a, bcs[a]);
    for (int a = 1; a < 3; ++a)
        if (bcs[a] != LBM_BC_PERIODIC && bcs[a] != LBM_BC_WALL)
            return fail(LBM_EINVAL, "inlet / outlet faces (Zou-He, anti-bounce-back, velocity) are on the x axis only");
    const bool faces = p->bc_x == LBM_BC_PRESSURE || p->bc_x == LBM_BC_ABB || p->bc_x == LBM_BC_VELOCITY;
    if (p->collision != LBM_COLL_BGK && p->collision != LBM_COLL_MRT) return fail(LBM_EINVAL, "bad collision");
    if (p->collision == LBM_COLL_MRT) {
        if (p->lattice != LBM_D2Q9) return fail(LBM_EINVAL, "the MRT collision is implemented for D2Q9 only");
        for (int r = 0; r < 7; ++r)
            if (!(p->mrt_rates[r] > 0.0 && p->mrt_rates[r] < 2.0))
                return fail(LBM_EINVAL, "MRT rate %d must lie in (0, 2) (got %g)", r, p->mrt_rates[r]);
    }
    if (p->steps < 1) return fail(LBM_EINVAL, "steps must be >= 1 (got %d)", p->steps);
    if (p->ckpt_interval < 0) return fail(LBM_EINVAL, "ckpt_interval must be >= 0");
    if (p->loss_kind != LBM_LOSS_VEC && p->loss_kind != LBM_LOSS_NORM) return fail(LBM_EINVAL, "bad loss_kind");
    if (p->loss_scale != LBM_SCALE_SUM && p->loss_scale != LBM_SCALE_MEAN_FLUID)
        return fail(LBM_EINVAL, "bad loss_scale");
    if (p->inlet_mode != LBM_INLET_CONST && p->inlet_mode != LBM_INLET_PROFILE)
        return fail(LBM_EINVAL, "bad inlet_mode");
    for (int b = 0; b < p->n_inst; ++b) {
        const lbm_instance &I = p->inst[b];
        if (I.nx < 1 || I.ny < 1 || I.nz < 1)
            return fail(LBM_EINVAL, "instance %d: dimensions must be positive (%d x %d x %d)", b, I.nx, I.ny, I.nz);
        if (p->lattice == LBM_D2Q9 && I.nz != 1) return fail(LBM_EINVAL, "instance %d: D2Q9 needs nz = 1", b);
        if (I.nx >= (1 << lbm::X_BITS))
            return fail(LBM_EINVAL, "instance %d: nx must be below %d (got %d)", b, 1 << lbm::X_BITS, I.nx);
        if (faces && I.nx < 2)
            return fail(LBM_EINVAL, "instance %d: density faces on x need nx >= 2", b);
        if ((long long)I.nx * I.ny * I.nz * p->lattice >= (1LL << 31) - (1LL << 20))
            return fail(LBM_EINVAL, "instance %d: Q x nodes must stay below 2^31 (32-bit population offsets)", b);
        const long long plane = std::max(64LL, (count_fluid(I) + 63) / 64 * 64);
        if ((long long)p->lattice * plane * 4 > MAX_INSTANCE_STATE_BYTES)
            return fail(LBM_EINVAL, "instance %d: Q x fluid nodes x 4 B must stay below 4 GiB per state "
                                    "(%lld padded fluid nodes)", b, plane);
        if (p->inlet_mode == LBM_INLET_PROFILE && faces && I.solid) {
            for (long long zy = 0; zy < (long long)I.ny * I.nz; ++zy)
                if (I.solid[zy * I.nx])
                    return fail(LBM_EINVAL, "instance %d: solid node on the inlet face in profile mode", b);
        }
    }
    return LBM_OK;
}

long long count_fluid(const lbm_instance &S) {
    const long long n = (long long)S.nx * S.ny * S.nz;
    if (!S.solid) return n;
    long long c = 0;
    for (long long k = 0; k < n; ++k) c += S.solid[k] == 0;
    return c;
}

void plan(const lbm_problem *p, Layout &L) {
    L.q = p->lattice;
    L.D = L.q == 9 ? 2 : 3;
    L.n_inst = p->n_inst;
    L.T = p->steps;
    L.K = p->ckpt_interval > 0 ? p->ckpt_interval : (int)ceil(sqrt((double)p->steps));
    if (L.K > L.T) L.K = L.T;
    L.n_seg = (L.T + L.K - 1) / L.K;
    L.tape = p->tape ? 1 : 0;
    L.R = std::min(std::max(p->resident_segments, 1), L.n_seg);
    L.frames = std::max(p->loss_frames, 1);
    L.stride = L.frames > 1 ? p->loss_stride : 1;
    L.inst.assign(p->n_inst, InstDev{});
    long long poff = 0, node = 0, face = 0, words = 0;
    int tile = 0, ftile = 0;
    for (int b = 0; b < p->n_inst; ++b) {
        const lbm_instance &S = p->inst[b];
        InstDev &I = L.inst[b];
        I.nx = S.nx; I.ny = S.ny; I.nz = S.nz;
        I.words = (S.nx + 31) / 32;
        I.tiles_x = (S.nx + lbm::TILE_X - 1) / lbm::TILE_X;
        I.tiles_y = (S.ny + lbm::TILE_Y - 1) / lbm::TILE_Y;
        I.n_tiles = I.tiles_x * I.tiles_y * S.nz;
        I.tile_begin = tile;
        tile += I.n_tiles;
        I.n_fluid = (int)count_fluid(S);
        I.n_ftiles = (I.n_fluid + lbm::FT - 1) / lbm::FT;
        I.ftile_begin = ftile;
        ftile += I.n_ftiles;
        // one plane per population direction over the fluid nodes, padded to 256 B
        I.plane = std::max<long long>(64, (long long)align_up((size_t)I.n_fluid, 64));
        I.poff = poff;
        I.st_off = (long long)L.q * poff;
        poff += I.plane;
        I.node_off = node;
        node += (long long)S.nx * S.ny * S.nz;
        I.face_off = face;
        face += (long long)S.ny * S.nz;
        I.rw_off = words;
        words += (long long)S.nz * S.ny * I.words;
        I.omega = 1.0f;
        I.inv_tau2 = 1.0f;
        I.loss_scale = 1.0f;
    }
    L.n_tiles = tile;
    L.n_ftiles = ftile;
    L.total_poff = poff;
    L.total_nodes = node;
    L.total_face = face;
    L.total_words = words;
    L.S = (long long)L.q * poff;
    L.n_states = 3 + (L.tape ? (L.n_seg - 1) + L.R * (L.K - 1) + 2 : 0);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
    L.off_inst = take(sizeof(InstDev) * p->n_inst);
    L.off_mask = take(sizeof(uint2) * words);
    L.off_roi = take(sizeof(float) * poff);
    L.off_target = take(sizeof(float) * poff * L.D * L.frames);
    L.off_face_in = take(sizeof(float) * face);
    L.off_face_out = take(sizeof(float) * face);
    L.off_grad_in = take(sizeof(double) * face);
    L.off_grad_out = take(sizeof(double) * face);
    L.off_part_loss = take(sizeof(double) * L.n_tiles);
    L.off_part_dtau = take(sizeof(double) * std::max(1, L.n_ftiles));
    L.off_part_res = take(sizeof(double) * 2 * L.n_tiles);
    L.off_red = take(sizeof(double) * 2 * p->n_inst);
    L.off_fblk = take(sizeof(lbm::FTileDesc) * std::max(1, L.n_ftiles));
    L.off_u2 = take(sizeof(float) * node * L.D);
    L.off_seed = take(sizeof(float) * node * L.D);
    L.off_flag = take(sizeof(unsigned));
    L.state_bytes = align_up(sizeof(float) * (size_t)L.S, 256);
    L.off_states = o;
    L.total = L.off_states + L.state_bytes * (size_t)L.n_states;
}

}  // namespace

struct lbm_handle {
    Layout L;
    lbm_problem P;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    lbm::Geo G{};
    std::vector<InstDev> hinst;
    std::vector<float> h_face_in, h_face_out;
    std::vector<double> h_red, h_grad;
    std::vector<double> res_last;     // per-instance residuals of the last residual check
    // state bookkeeping
    float *cur = nullptr, *prev = nullptr;
    long long cur_steps = 0;          // steps taken since the initial state
    bool fwd_taped = false, adjoint_done = false, resident_valid = false;
    float *nu_last = nullptr;         // nu^1 after the adjoint
    std::vector<double> tau;          // parameters of the taped forward
    // timing
    bool timing = false;
    lbm_timing tm{};
    std::vector<hipEvent_t> ev;
    // graphs: captured on a private stream, launched on the caller's stream
    bool graphs = true;
    hipStream_t cap = nullptr;
    hipGraphExec_t g_fwd[2] = {nullptr, nullptr};            // [record_tape]
    hipGraphExec_t g_rev[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [!resident][seed]
    hipGraphExec_t g_chunk[2] = {nullptr, nullptr};          // [starts from the initial state]
    int chunk_len = 0;
    // reverse sweep with recompute beside the adjoint: a second stream and its events
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> xev;

    float *state(int k) const { return (float *)(ws + L.off_states + L.state_bytes * (size_t)k); }
    float *init() const { return state(0); }
    float *pp(int k) const { return state(1 + k); }
    float *ckpt(int c) const { return c == 0 ? init() : state(3 + (c - 1)); }
    // state j (1 .. K-1) of segment region r (0 .. R-1); region r holds segment n_seg - R + r
    // after a taped forward; the reverse sweep recomputes the other segments into region 0,
    // or into regions 0 and 1 in turn when the recompute runs beside the adjoint
    float *seg(int r, int j) const { return state(3 + (L.n_seg - 1) + r * (L.K - 1) + (j - 1)); }
    float *nu(int k) const { return state(3 + (L.n_seg - 1) + L.R * (L.K - 1) + k); }
    template <class T> T *at(size_t off) const { return (T *)(ws + off); }
};

namespace {

int upload_params(lbm_handle *h, const lbm_params *prm) {
    if (!prm || !prm->tau || !prm->drho_in || !prm->drho_out)
        return fail(LBM_EINVAL, "params and their tau, drho_in, drho_out arrays must be non-NULL");
    const Layout &L = h->L;
    h->h_face_in.assign(L.total_face, 0.f);
    h->h_face_out.assign(L.total_face, 0.f);
    long long prof = 0;
    for (int b = 0; b < L.n_inst; ++b) {
        InstDev &I = h->hinst[b];
        const double tau = prm->tau[b];
        if (!(tau > 0.5) || !isfinite(tau)) return fail(LBM_EINVAL, "instance %d: tau must be > 0.5 (got %g)", b, tau);
        I.omega = (float)(1.0 / tau);
        I.inv_tau2 = (float)(1.0 / (tau * tau));
        const long long nf = (long long)I.ny * I.nz;
        const double dout = prm->drho_out[b];
        if (!isfinite(dout) || dout <= -1.0) return fail(LBM_EINVAL, "instance %d: drho_out must be finite and > -1", b);
        for (long long k = 0; k < nf; ++k) {
            double din = h->P.inlet_mode == LBM_INLET_PROFILE ? prm->drho_in[prof + k] : prm->drho_in[b];
            if (h->P.bc_x == LBM_BC_VELOCITY) {
                if (!isfinite(din) || !(din > -1.0 && din < 1.0))
                    return fail(LBM_EINVAL, "instance %d: inlet velocity must lie in (-1, 1)", b);
            } else if (!isfinite(din) || din <= -1.0) {
                return fail(LBM_EINVAL, "instance %d: drho_in must be finite and > -1", b);
            }
            h->h_face_in[I.face_off + k] = (float)din;
            h->h_face_out[I.face_off + k] = (float)dout;
        }
        prof += nf;
    }
    HIP_TRY(hipMemcpyAsync(h->at<InstDev>(L.off_inst), h->hinst.data(), sizeof(InstDev) * L.n_inst,
                           hipMemcpyHostToDevice, h->stream));
    if (L.total_face) {
        HIP_TRY(hipMemcpyAsync(h->at<float>(L.off_face_in), h->h_face_in.data(), sizeof(float) * L.total_face,
                               hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(h->at<float>(L.off_face_out), h->h_face_out.data(),
                               sizeof(float) * L.total_face, hipMemcpyHostToDevice, h->stream));
    }
    return LBM_OK;
}

int record(lbm_handle *h, int idx) {
    if (!h->timing) return LBM_OK;
    while ((int)h->ev.size() <= idx) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        h->ev.push_back(e);
    }
    HIP_TRY(hipEventRecord(h->ev[idx], h->stream));
    return LBM_OK;
}

double elapsed(lbm_handle *h, int a, int b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev[a], h->ev[b]);
    return ms;
}

// tape: dst is a tape state (a checkpoint or a segment state), read again
// only by the reverse sweep, long after it would have left the cache.
int step(lbm_handle *h, const float *src, float *dst, hipStream_t s, bool tape = false) {
    HIP_TRY(lbm::launch_step(h->L.q, h->G, src, dst, h->at<float>(h->L.off_face_in),
                             h->at<float>(h->L.off_face_out), tape, s));
    return LBM_OK;
}

// Runs `enqueue(stream)` either directly on the caller's stream or, with
// graphs enabled, as a hipGraph captured once (on a private stream) and
// replayed on the caller's stream.  Every pointer the enqueued work uses is
// fixed for the life of the handle and parameters live in device memory, so
// a captured graph stays valid.
template <class F>
int with_graph(lbm_handle *h, hipGraphExec_t &slot, F &&enqueue) {
    if (!h->graphs) return enqueue(h->stream);
    if (!slot) {
        if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        int rc = enqueue(h->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(h->cap, &g);
        if (rc) {
            if (e == hipSuccess && g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(LBM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&slot, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            slot = nullptr;
            return fail(LBM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        }
    }
    HIP_TRY(hipGraphLaunch(slot, h->stream));
    return LBM_OK;
}

int reduce_to_host(lbm_handle *h, size_t part_off, int stride, int fluid) {
    const Layout &L = h->L;
    HIP_TRY(lbm::launch_reduce(h->at<InstDev>(L.off_inst), L.n_inst, h->at<double>(part_off), stride, fluid,
                               h->at<double>(L.off_red), h->stream));
    h->h_red.assign((size_t)L.n_inst * stride, 0.0);
    HIP_TRY(hipMemcpyAsync(h->h_red.data(), h->at<double>(L.off_red), sizeof(double) * L.n_inst * stride,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

const char *lbm_strerror(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "workspace too small";
        case LBM_ESTATE: return "call out of order";
        case LBM_EUNSTABLE: return "non-finite value (unstable run)";
        case LBM_ECORRUPT: return "recomputed state does not match its checkpoint";
        case LBM_EDEVICE: return "HIP runtime error";
        default: return "unknown error";
    }
}

const char *lbm_last_error(void) { return g_err.c_str(); }

int lbm_workspace_bytes(const lbm_problem *p, size_t *bytes) {
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    Layout L;
    plan(p, L);
    *bytes = L.total;
    return LBM_OK;
}

int lbm_init(lbm_handle **out, const lbm_problem *p, void *d_workspace, size_t bytes, void *hip_stream) {
    if (!out) return fail(LBM_EINVAL, "handle pointer is NULL");
    *out = nullptr;
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!d_workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_workspace) & 255) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    lbm_handle *h = new lbm_handle();
    plan(p, h->L);
    if (bytes < h->L.total) {
        size_t need = h->L.total;
        delete h;
        return fail(LBM_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
    }
    h->P = *p;
    h->P.inst = nullptr;
    h->stream = (hipStream_t)hip_stream;
    h->ws = (char *)d_workspace;
    h->hinst = h->L.inst;
    const Layout &L = h->L;
    // host copies of the row-word tables, weights and targets in the device layouts
    std::vector<uint2> rw(L.total_words);
    const size_t frame_floats = (size_t)L.total_poff * L.D;
    std::vector<float> roi(L.total_poff, 0.f), target(frame_floats * L.frames, 0.f);
    for (int b = 0; b < L.n_inst; ++b) {
        const lbm_instance &S = p->inst[b];
        InstDev &I = h->hinst[b];
        long long id = 0;
        for (int z = 0; z < S.nz; ++z)
            for (int y = 0; y < S.ny; ++y)
                for (int w = 0; w < I.words; ++w) {
                    uint2 &e = rw[I.rw_off + ((long long)z * S.ny + y) * I.words + w];
                    e.x = 0u;
                    e.y = (uint32_t)id;
                    for (int bit = 0; bit < 32; ++bit) {
                        const int x = 32 * w + bit;
                        const long long dn = ((long long)z * S.ny + y) * S.nx + x;
                        if (x >= S.nx || (S.solid && S.solid[dn])) {
                            e.x |= 1u << bit;
                            continue;
                        }
                        roi[I.poff + id] = S.roi ? S.roi[dn] : 1.0f;
                        if (S.target_u)
                            for (int f = 0; f < L.frames; ++f) {
                                const long long fdn = (long long)f * S.nz * S.ny * S.nx + dn;
                                for (int a = 0; a < L.D; ++a)
                                    target[f * frame_floats + I.poff * L.D + a * I.plane + id] =
                                        S.target_u[fdn * L.D + a];
                            }
                        ++id;
                    }
                }
        I.loss_scale = p->loss_scale == LBM_SCALE_MEAN_FLUID ? (id ? (float)(1.0 / (double)id) : 0.f) : 1.0f;
    }
    // per fluid tile: the instance-local row words holding its first and last fluid id
    std::vector<lbm::FTileDesc> fblk(std::max(1, L.n_ftiles), lbm::FTileDesc{});
    for (int b = 0; b < L.n_inst; ++b) {
        const InstDev &I = h->hinst[b];
        const long long nw = (long long)I.nz * I.ny * I.words;
        long long w = 0;
        for (int t = 0; t < I.n_ftiles; ++t) {
            const long long first = (long long)t * lbm::FT;
            const long long last = std::min<long long>(first + lbm::FT, I.n_fluid) - 1;
            lbm::FTileDesc &e = fblk[I.ftile_begin + t];
            e.b = b;
            // word holding id k: the last word whose first id is <= k and that has a fluid node
            auto holds = [&](long long ww, long long k) {
                const uint2 r = rw[I.rw_off + ww];
                const long long nf = __builtin_popcount(~r.x);
                return (long long)r.y <= k && k < (long long)r.y + nf;
            };
            while (w < nw && !holds(w, first)) ++w;
            e.w0 = (int)w;
            long long w1 = w;
            while (w1 < nw && !holds(w1, last)) ++w1;
            e.w1 = (int)w1;
            e.r0 = (int)(w / I.words);
            e.r1 = (int)(w1 / I.words);
        }
    }
    auto cp = [&](size_t off, const void *src, size_t n) -> int {
        if (!n) return LBM_OK;
        HIP_TRY(hipMemcpyAsync(h->ws + off, src, n, hipMemcpyHostToDevice, h->stream));
        return LBM_OK;
    };
    int e = 0;
    if ((e = cp(L.off_inst, h->hinst.data(), sizeof(InstDev) * L.n_inst)) ||
        (e = cp(L.off_mask, rw.data(), sizeof(uint2) * rw.size())) ||
        (e = cp(L.off_fblk, fblk.data(), sizeof(lbm::FTileDesc) * fblk.size())) ||
        (e = cp(L.off_roi, roi.data(), sizeof(float) * roi.size())) ||
        (e = cp(L.off_target, target.data(), sizeof(float) * target.size()))) {
        delete h;
        return e;
    }
    h->G.inst = h->at<InstDev>(L.off_inst);
    h->G.n_inst = L.n_inst;
    h->G.n_tiles = L.n_tiles;
    h->G.bcx = p->bc_x; h->G.bcy = p->bc_y; h->G.bcz = p->bc_z;
    h->G.coll = p->collision;
    for (int r = 0; r < 9; ++r) h->G.mrt[r] = (float)p->mrt_rates[r];
    h->G.rw = h->at<uint2>(L.off_mask);
    h->G.n_ftiles = L.n_ftiles;
    // a step reads one state and writes another: when the two exceed the
    // 256 MiB Infinity Cache the written lines only evict what the next step
    // reads, so step and adjoint stores go out non-temporal
    h->G.nt = 2 * L.state_bytes > ((size_t)256 << 20);
    h->G.fblk = h->at<lbm::FTileDesc>(L.off_fblk);
    hipError_t he = lbm::launch_init_eq(L.q, h->G, h->init(), nullptr, nullptr, h->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(h->stream);
    if (he != hipSuccess) {
        delete h;
        return fail(LBM_EDEVICE, "initial state: %s", hipGetErrorString(he));
    }
    h->cur = h->init();
    h->prev = nullptr;
    h->cur_steps = 0;
    *out = h;
    return LBM_OK;
}

int lbm_destroy(lbm_handle *h) {
    if (!h) return LBM_OK;
    for (auto e : h->ev) (void)hipEventDestroy(e);
    for (auto g : h->g_fwd) if (g) (void)hipGraphExecDestroy(g);
    for (auto &r : h->g_rev) for (auto g : r) if (g) (void)hipGraphExecDestroy(g);
    for (auto g : h->g_chunk) if (g) (void)hipGraphExecDestroy(g);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->side) (void)hipStreamDestroy(h->side);
    for (auto e : h->xev) (void)hipEventDestroy(e);
    delete h;
    return LBM_OK;
}

static void reset_state(lbm_handle *h) {
    h->cur = h->init();
    h->prev = nullptr;
    h->cur_steps = 0;
    h->fwd_taped = h->adjoint_done = h->resident_valid = false;
}

int lbm_set_initial(lbm_handle *h, const float *d_drho, const float *d_u) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    HIP_TRY(lbm::launch_init_eq(h->L.q, h->G, h->init(), d_drho, d_u, h->stream));
    reset_state(h);
    return LBM_OK;
}

int lbm_set_populations(lbm_handle *h, const float *d_fbar) {
    if (!h || !d_fbar) return fail(LBM_EINVAL, "handle and populations must be non-NULL");
    HIP_TRY(lbm::launch_convert(h->L.q, h->G, h->init(), (float *)d_fbar, 1, h->stream));
    reset_state(h);
    return LBM_OK;
}

int lbm_get_populations(lbm_handle *h, int which, float *d_out) {
    if (!h || !d_out) return fail(LBM_EINVAL, "handle and output must be non-NULL");
    if (which == LBM_POP_STATE) {
        HIP_TRY(lbm::launch_convert(h->L.q, h->G, h->cur, d_out, 0, h->stream));
        return LBM_OK;
    }
    if (which == LBM_POP_ADJOINT) {
        if (!h->adjoint_done) return fail(LBM_ESTATE, "no adjoint has been computed");
        HIP_TRY(lbm::launch_adj_final(h->L.q, h->G, h->nu_last, h->init(), h->at<float>(h->L.off_face_in),
                                      h->at<float>(h->L.off_face_out), d_out, h->L.total_nodes * h->L.q,
                                      h->stream));
        return LBM_OK;
    }
    return fail(LBM_EINVAL, "unknown population kind %d", which);
}

// Destination of step t of the forward pass.  With a tape, F^{cK} goes to
// checkpoint c and the states of the last R segments go straight to their
// regions of the segment store, so the reverse sweep does not recompute them.
static float *fwd_dst(lbm_handle *h, int t, int record_tape) {
    const Layout &L = h->L;
    if (record_tape && t < L.T) {
        const int c = t / L.K, j = t % L.K, r = c - (L.n_seg - L.R);
        return j == 0 ? h->ckpt(c) : (r >= 0 ? h->seg(r, j) : h->pp(t & 1));
    }
    return h->pp(t & 1);
}

// Loss frame of the state after step t, or -1: frames sit at
// T - (frames - 1 - m) stride, m = 0 .. frames - 1.
static int frame_of(const Layout &L, int t) {
    const int back = L.T - t;
    if (back < 0 || back % L.stride) return -1;
    const int m = L.frames - 1 - back / L.stride;
    return m >= 0 ? m : -1;
}

static const float *frame_target(lbm_handle *h, int m) {
    return h->at<float>(h->L.off_target) + (size_t)m * h->L.total_poff * h->L.D;
}

// The steps of a forward pass; the frames of a time-windowed loss before T
// add their partial sums as the pass goes (the frame at T is added by
// lbm_forward when a loss is asked for).
static int enqueue_forward(lbm_handle *h, int record_tape, hipStream_t s) {
    const Layout &L = h->L;
    const float *src = h->init();
    for (int t = 1; t <= L.T; ++t) {
        float *dst = fwd_dst(h, t, record_tape);
        int rc = step(h, src, dst, s, dst != h->pp(0) && dst != h->pp(1));
        if (rc) return rc;
        const int m = t < L.T ? frame_of(L, t) : -1;
        if (m >= 0)
            HIP_TRY(lbm::launch_loss(L.q, h->G, dst, h->at<float>(L.off_roi), frame_target(h, m), h->P.loss_kind,
                                     h->at<double>(L.off_part_loss), m > 0, s));
        src = dst;
    }
    return LBM_OK;
}

int lbm_forward(lbm_handle *h, const lbm_params *prm, int record_tape, double *loss_out) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    const Layout &L = h->L;
    if (record_tape && !L.tape) return fail(LBM_ESTATE, "the problem was planned without a tape");
    int rc = upload_params(h, prm);
    if (rc) return rc;
    record_tape = record_tape ? 1 : 0;
    h->fwd_taped = h->adjoint_done = false;
    const int T = L.T;
    if ((rc = record(h, 0))) return rc;
    if (h->timing) rc = enqueue_forward(h, record_tape, h->stream);
    else rc = with_graph(h, h->g_fwd[record_tape], [&](hipStream_t s) { return enqueue_forward(h, record_tape, s); });
    if (rc) return rc;
    if ((rc = record(h, 1))) return rc;
    h->cur = fwd_dst(h, T, record_tape);
    h->prev = T >= 2 ? fwd_dst(h, T - 1, record_tape) : h->init();
    h->cur_steps = T;
    if (record_tape) {
        h->fwd_taped = true;
        h->resident_valid = true;
        h->tau.assign(prm->tau, prm->tau + L.n_inst);
    }
    if (loss_out) {
        HIP_TRY(lbm::launch_loss(L.q, h->G, h->cur, h->at<float>(L.off_roi), frame_target(h, L.frames - 1),
                                 h->P.loss_kind, h->at<double>(L.off_part_loss), L.frames > 1, h->stream));
        if ((rc = reduce_to_host(h, L.off_part_loss, 1, 0))) return rc;
        bool finite = true;
        for (int b = 0; b < L.n_inst; ++b) {
            loss_out[b] = h->h_red[b];
            finite = finite && isfinite(h->h_red[b]);
        }
        if (!finite) return fail(LBM_EUNSTABLE, "non-finite loss after %d steps", T);
    }
    if (h->timing) {
        HIP_TRY(hipEventSynchronize(h->ev[1]));
        h->tm.forward_ms += elapsed(h, 0, 1);
        h->tm.forward_launches += T;
    }
    return LBM_OK;
}

// The reverse sweep: zero the accumulators, then per segment (last first)
// recompute its states from the checkpoint and run the adjoint steps.  While
// the taped forward's states are intact (resident), the last R segments are
// read from their own regions; every other segment is recomputed into a
// region whose resident states have been consumed by then (region 0, or
// regions 0 and 1 in turn when R >= 2 lets the recompute run beside the
// adjoint).  Event marks (timing mode only) bracket each segment's two
// phases, with the segments in sequence.
static int enqueue_reverse(lbm_handle *h, bool resident, const float *seed, hipStream_t s,
                           std::vector<int> *marks) {
    const Layout &L = h->L;
    const int q = L.q, T = L.T, K = L.K;
    HIP_TRY(lbm::launch_fill_f64(h->at<double>(L.off_grad_in), L.total_face, 0.0, s));
    HIP_TRY(lbm::launch_fill_f64(h->at<double>(L.off_grad_out), L.total_face, 0.0, s));
    HIP_TRY(lbm::launch_fill_f64(h->at<double>(L.off_part_dtau), L.n_ftiles, 0.0, s));
    const float *fin = h->at<float>(L.off_face_in), *fout = h->at<float>(L.off_face_out);
    double *gin = h->at<double>(L.off_grad_in), *gout = h->at<double>(L.off_grad_out);
    double *dpart = h->at<double>(L.off_part_dtau);
    unsigned *flag = h->at<unsigned>(L.off_flag);
    HIP_TRY(lbm::launch_fill_u32(flag, 1, 0u, s));
    const int n_seg = L.n_seg;
    int ev = 0, rc;
    // adjoint steps of segment c, reading its states from region r
    auto adjoint_segment = [&](int c, int r, hipStream_t st) -> int {
        const int t0 = c * K, t1 = std::min(t0 + K, T);
        for (int k = t1; k > t0; --k) {
            const float *Fprev = k - 1 - t0 == 0 ? h->ckpt(c) : h->seg(r, k - 1 - t0);
            float *nu_out = h->nu(k & 1);
            if (k == T) {
                HIP_TRY(lbm::launch_adj_seed(q, h->G, Fprev, nu_out, fin, fout, gin, gout,
                                             h->at<float>(L.off_roi), frame_target(h, L.frames - 1),
                                             h->P.loss_kind, seed, st));
            } else {
                const int m = frame_of(L, k);
                HIP_TRY(lbm::launch_adj_step(q, h->G, Fprev, h->nu((k + 1) & 1), nu_out, fin, fout, gin, gout,
                                             dpart, h->at<float>(L.off_roi), m >= 0 ? frame_target(h, m) : nullptr,
                                             h->P.loss_kind, st));
            }
        }
        return LBM_OK;
    };
    // Recomputes segment c into region r; a segment followed by a checkpoint
    // then takes one more step with the same kernel into a scratch state (the
    // ping-pong buffer that does not hold F^T), compared bit for bit with
    // that checkpoint (a mismatch raises the flag that lbm_grad reports).
    float *scratch = h->pp(1 - (T & 1));
    auto recompute_segment = [&](int c, int r, hipStream_t st) -> int {
        const int t0 = c * K, t1 = std::min(t0 + K, T);
        for (int j = 1; j < t1 - t0; ++j)
            if ((rc = step(h, j == 1 ? h->ckpt(c) : h->seg(r, j - 1), h->seg(r, j), st, true))) return rc;
        if (c + 1 < n_seg) {
            if ((rc = step(h, t1 - t0 > 1 ? h->seg(r, t1 - t0 - 1) : h->ckpt(c), scratch, st))) return rc;
            HIP_TRY(lbm::launch_compare(q, h->G, scratch, h->ckpt(c + 1), flag, st));
        }
        return LBM_OK;
    };
    auto kept = [&](int k) { return resident && k < L.R; };          // k-th segment of the sweep, c = n_seg - 1 - k
    if (!marks && L.R >= 2 && !kept(n_seg - 1)) {
        // Recompute beside the adjoint: the k-th segment of the sweep is recomputed on a second
        // stream into region(k) while the adjoint consumes segment k - 1.  Kept segments read
        // their own regions R - 1 - k; the others alternate between the two regions whose
        // adjoint finished two segments earlier (region(k) = region(k - 2)), so a recompute
        // never overwrites states that an adjoint still reads.
        std::vector<int> region(n_seg);
        for (int k = 0; k < n_seg; ++k) region[k] = kept(k) ? L.R - 1 - k : (k >= 2 ? region[k - 2] : k);
        if (!h->side) HIP_TRY(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        while ((int)h->xev.size() < 2 * n_seg + 1) {
            hipEvent_t e;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            h->xev.push_back(e);
        }
        hipEvent_t fork = h->xev[2 * n_seg];
        auto rec_done = [&](int k) { return h->xev[2 * k]; };
        auto adj_done = [&](int k) { return h->xev[2 * k + 1]; };
        HIP_TRY(hipEventRecord(fork, s));
        HIP_TRY(hipStreamWaitEvent(h->side, fork, 0));
        auto issue_recompute = [&](int k) -> int {
            if (k >= 2) HIP_TRY(hipStreamWaitEvent(h->side, adj_done(k - 2), 0));
            if ((rc = recompute_segment(n_seg - 1 - k, region[k], h->side))) return rc;
            HIP_TRY(hipEventRecord(rec_done(k), h->side));
            return LBM_OK;
        };
        for (int k = 0; k < n_seg; ++k) {
            if (k == 0 && !kept(0) && (rc = issue_recompute(0))) return rc;
            if (k + 1 < n_seg && !kept(k + 1) && (rc = issue_recompute(k + 1))) return rc;
            if (!kept(k)) HIP_TRY(hipStreamWaitEvent(s, rec_done(k), 0));
            if ((rc = adjoint_segment(n_seg - 1 - k, region[k], s))) return rc;
            HIP_TRY(hipEventRecord(adj_done(k), s));
        }
    } else {
        for (int c = n_seg - 1; c >= 0; --c) {
            const int t0 = c * K, t1 = std::min(t0 + K, T);
            const bool keep = resident && c >= n_seg - L.R;
            const int r = keep ? c - (n_seg - L.R) : 0;
            if (marks) { if ((rc = record(h, ev))) return rc; marks->push_back(ev++); }
            if (!keep) {
                if ((rc = recompute_segment(c, r, s))) return rc;
                if (marks) h->tm.recompute_launches += t1 - t0 - 1 + (c + 1 < n_seg ? 1 : 0);
            }
            if (marks) { if ((rc = record(h, ev))) return rc; marks->push_back(ev++); }
            if ((rc = adjoint_segment(c, r, s))) return rc;
            if (marks) { if ((rc = record(h, ev))) return rc; marks->push_back(ev++); }
        }
    }
    // anti-bounce-back: the faces' density also entered g^1, through F^0
    if (L.T >= 1 && h->P.bc_x == LBM_BC_ABB)
        HIP_TRY(lbm::launch_abb_grad0(q, h->G, h->init(), h->nu(1), fin, fout, gin, gout, s));
    return LBM_OK;
}

int lbm_adjoint(lbm_handle *h, const float *d_seed_du) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (!h->fwd_taped) return fail(LBM_ESTATE, "lbm_adjoint needs a preceding lbm_forward with record_tape");
    const Layout &L = h->L;
    int rc;
    const float *seed = nullptr;
    if (d_seed_du && L.frames > 1)
        return fail(LBM_EINVAL, "a caller seed replaces the loss at T only; loss_frames > 1 needs the built-in loss");
    if (d_seed_du) {
        // a fixed internal copy keeps captured graphs valid for any caller buffer
        HIP_TRY(hipMemcpyAsync(h->at<float>(L.off_seed), d_seed_du, sizeof(float) * L.total_nodes * L.D,
                               hipMemcpyDeviceToDevice, h->stream));
        seed = h->at<float>(L.off_seed);
    }
    const bool resident = h->resident_valid;
    if (h->timing) {
        std::vector<int> marks;
        if ((rc = enqueue_reverse(h, resident, seed, h->stream, &marks))) return rc;
        HIP_TRY(hipEventSynchronize(h->ev[marks.back()]));
        for (int c = L.n_seg - 1, k = 0; c >= 0; --c, k += 3) {
            const int t0 = c * L.K, t1 = std::min(t0 + L.K, L.T);
            h->tm.recompute_ms += elapsed(h, marks[k], marks[k + 1]);
            h->tm.adjoint_ms += elapsed(h, marks[k + 1], marks[k + 2]);
            h->tm.adjoint_launches += t1 - t0;
        }
    } else {
        rc = with_graph(h, h->g_rev[resident ? 0 : 1][seed ? 1 : 0],
                        [&](hipStream_t s) { return enqueue_reverse(h, resident, seed, s, nullptr); });
        if (rc) return rc;
    }
    // recomputed segments overwrite regions 0 and 1; with every segment resident nothing is recomputed
    h->resident_valid = (resident && L.R == L.n_seg) || L.n_seg == 1;
    h->nu_last = h->nu(1);
    h->adjoint_done = true;
    h->prev = nullptr;  // the segment store that held F^{T-1} has been reused
    return LBM_OK;
}

int lbm_grad(lbm_handle *h, double *d_rho_in, double *d_tau, double *d_rho_out) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (!h->adjoint_done) return fail(LBM_ESTATE, "lbm_grad needs a preceding lbm_adjoint");
    const Layout &L = h->L;
    unsigned corrupt = 0;
    HIP_TRY(hipMemcpyAsync(&corrupt, h->at<unsigned>(L.off_flag), sizeof(unsigned), hipMemcpyDeviceToHost,
                           h->stream));
    int rc = reduce_to_host(h, L.off_part_dtau, 1, 1);
    if (rc) return rc;
    if (corrupt)
        return fail(LBM_ECORRUPT, "a segment recomputed by the reverse sweep did not reproduce the next "
                                  "checkpoint bit for bit (tape memory overwritten, or a non-deterministic step)");
    std::vector<double> gin(L.total_face), gout(L.total_face);
    if (L.total_face) {
        HIP_TRY(hipMemcpyAsync(gin.data(), h->at<double>(L.off_grad_in), sizeof(double) * L.total_face,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(gout.data(), h->at<double>(L.off_grad_out), sizeof(double) * L.total_face,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    long long prof = 0;
    bool finite = true;
    for (int b = 0; b < L.n_inst; ++b) {
        const InstDev &I = h->hinst[b];
        const long long nf = (long long)I.ny * I.nz;
        double si = 0.0, so = 0.0;
        for (long long k = 0; k < nf; ++k) {
            si += gin[I.face_off + k];
            so += gout[I.face_off + k];
            if (d_rho_in && h->P.inlet_mode == LBM_INLET_PROFILE) d_rho_in[prof + k] = gin[I.face_off + k];
        }
        if (d_rho_in && h->P.inlet_mode == LBM_INLET_CONST) d_rho_in[b] = si;
        if (d_rho_out) d_rho_out[b] = so;
        if (d_tau) d_tau[b] = h->h_red[b];
        finite = finite && isfinite(si) && isfinite(so) && isfinite(h->h_red[b]);
        prof += nf;
    }
    if (!finite) return fail(LBM_EUNSTABLE, "non-finite gradient");
    return LBM_OK;
}

// One residual chunk: check_every steps from src over the ping-pong
// buffers (pp0, pp1, pp0, ...), then the residual partial sums of the two-step
// mean of the last two states against the snapshot of the previous check
// (the first chunk takes the snapshot of the initial state first).
static int enqueue_chunk(lbm_handle *h, const float *src, bool first, int check_every, hipStream_t s) {
    const Layout &L = h->L;
    float *snap = h->at<float>(L.off_u2);
    if (first) HIP_TRY(lbm::launch_macro(L.q, h->G, src, nullptr, nullptr, snap, s));
    const float *prev = nullptr;
    for (int k = 0; k < check_every; ++k) {
        float *dst = h->pp(k & 1);
        int rc = step(h, src, dst, s);
        if (rc) return rc;
        prev = src;
        src = dst;
    }
    HIP_TRY(lbm::launch_residual(L.q, h->G, src, prev, snap, h->at<double>(L.off_part_res), s));
    HIP_TRY(lbm::launch_reduce(h->at<InstDev>(L.off_inst), L.n_inst, h->at<double>(L.off_part_res), 2, 0,
                               h->at<double>(L.off_red), s));
    return LBM_OK;
}

int lbm_run_to_residual(lbm_handle *h, const lbm_params *prm, double tol, int max_steps, int check_every,
                        int *steps_out, double *r_out) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (check_every < 4 || (check_every & 1)) return fail(LBM_EINVAL, "check_every must be even and >= 4");
    if (max_steps < check_every) return fail(LBM_EINVAL, "max_steps must be >= check_every");
    const Layout &L = h->L;
    int rc = upload_params(h, prm);
    if (rc) return rc;
    h->fwd_taped = h->adjoint_done = false;
    if (h->chunk_len != check_every) {
        for (auto &g : h->g_chunk)
            if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
        h->chunk_len = check_every;
    }
    int t = 0;
    double rmax = INFINITY;
    h->h_red.assign(2 * (size_t)L.n_inst, 0.0);
    while (t + check_every <= max_steps) {
        const float *src = t == 0 ? h->init() : h->pp(1);
        rc = with_graph(h, h->g_chunk[t == 0 ? 1 : 0],
                        [&](hipStream_t s) { return enqueue_chunk(h, src, t == 0, check_every, s); });
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(h->h_red.data(), h->at<double>(L.off_red), sizeof(double) * 2 * L.n_inst,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        t += check_every;
        h->cur = h->pp(1);
        h->prev = h->pp(0);
        rmax = 0.0;
        h->res_last.assign(L.n_inst, NAN);
        for (int b = 0; b < L.n_inst; ++b) {
            const double num = h->h_red[2 * b], den = h->h_red[2 * b + 1];
            if (!isfinite(num) || !isfinite(den)) {
                h->cur_steps = t;
                if (steps_out) *steps_out = t;
                if (r_out) *r_out = NAN;
                return fail(LBM_EUNSTABLE, "non-finite residual at step %d (instance %d)", t, b);
            }
            const double r = den > 0 ? sqrt(num / den) / check_every : (num > 0 ? INFINITY : 0.0);
            h->res_last[b] = r;
            rmax = std::max(rmax, r);
        }
        if (rmax <= tol) break;
    }
    h->cur_steps = t;
    if (steps_out) *steps_out = t;
    if (r_out) *r_out = rmax;
    return LBM_OK;
}

int lbm_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream) {
    if (!d_dst || !d_src) return fail(LBM_EINVAL, "pointers must be non-NULL");
    if ((bytes & 15) || (((uintptr_t)d_dst | (uintptr_t)d_src) & 15))
        return fail(LBM_EINVAL, "bytes and both pointers must be multiples of 16");
    HIP_TRY(lbm::launch_copy16(d_src, d_dst, (long long)(bytes / 16), (hipStream_t)hip_stream));
    return LBM_OK;
}

int lbm_get_residuals(lbm_handle *h, double *r_out) {
    if (!h || !r_out) return fail(LBM_EINVAL, "handle and output must be non-NULL");
    if (h->res_last.empty()) return fail(LBM_ESTATE, "no residual has been computed");
    std::copy(h->res_last.begin(), h->res_last.end(), r_out);
    return LBM_OK;
}

int lbm_set_graphs(lbm_handle *h, int enable) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    h->graphs = enable != 0;
    return LBM_OK;
}

int lbm_get_macro(lbm_handle *h, float *d_drho, float *d_u, int mean2) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (mean2 && (!h->prev || h->cur_steps < 2)) return fail(LBM_ESTATE, "mean of two states needs two steps");
    HIP_TRY(lbm::launch_macro(h->L.q, h->G, h->cur, mean2 ? h->prev : nullptr, d_drho, d_u, h->stream));
    return LBM_OK;
}

int lbm_checkpoint(lbm_handle *h, int c, void **d_state, size_t *bytes) {
    if (!h || !d_state) return fail(LBM_EINVAL, "handle and output must be non-NULL");
    if (!h->L.tape) return fail(LBM_ESTATE, "the problem was planned without a tape");
    if (c < 1 || c >= h->L.n_seg)
        return fail(LBM_EINVAL, "checkpoint %d is outside 1 .. %d", c, h->L.n_seg - 1);
    *d_state = h->ckpt(c);
    if (bytes) *bytes = sizeof(float) * (size_t)h->L.S;
    return LBM_OK;
}

int lbm_set_timing(lbm_handle *h, int enable, int reset) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    h->timing = enable != 0;
    if (reset) h->tm = lbm_timing{};
    return LBM_OK;
}

int lbm_get_timing(lbm_handle *h, lbm_timing *out) {
    if (!h || !out) return fail(LBM_EINVAL, "handle and output must be non-NULL");
    *out = h->tm;
    return LBM_OK;
}

}  // extern "C"
