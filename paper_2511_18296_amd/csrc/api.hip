// api.hip -- the extern "C" entry points declared in include/mps.h: argument
// checks, model ownership, workspaces and kernel launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"
#include "repair.h"
#include "internal.h"

using namespace mps;

namespace {

thread_local std::string g_err;

mps_status fail(mps_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

mps_status dev_fail(hipError_t e, const char *what) {
    return fail(MPS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Switch to a device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Device buffers owned by one mps_search call.
struct SearchBufs {
    std::vector<void *> ptrs;
    ~SearchBufs() {
        for (void *p : ptrs) hipFree(p);
    }
    template <class T>
    T *get(size_t count) {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(T) * (count > 0 ? count : 1)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        ptrs.push_back(p);
        return (T *)p;
    }
    // A workspace whose first `zero` bytes start zero (top-k and ranking
    // workspaces); nullptr if the allocation or the clearing fails.
    char *get_zeroed(size_t bytes, size_t zero, hipStream_t st) {
        char *p = get<char>(bytes);
        if (p && hipMemsetAsync(p, 0, zero < bytes ? zero : bytes, st) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
};

}  // namespace

// Status reporting for entry points defined in other translation units.
mps_status mps::report_error(mps_status st, const char *msg) {
    g_err = msg;
    return st;
}

struct mps_model {
    int device = 0;
    mps_params prm{};
    DevModel d{};
    std::vector<void *> allocs;
    size_t bytes = 0;
    size_t limit = 0;      // test-only allocation cap (0 = none)
    double *partial = nullptr;
    int chunks = 16;
    double *obj_dev = nullptr;   // double[7]
    void *relax_ws = nullptr;    // partial sums of the relaxed forward pass
    void *gather = nullptr;      // candidate records of a repair walk
    int32_t *rep_first = nullptr;   // [N] first candidate of each block in a walk; INT32_MAX between calls
    uint8_t *cmark = nullptr;       // [N] blocks moved in a cascading repair call
    double *wmult = nullptr;        // [S][T+1] discounted value multipliers (once set)
    float *wmult32 = nullptr;
    char *arena = nullptr;       // mutable search state (see mps_state_save)
    size_t arena_bytes = 0;
    int max_lds = 65536;

    template <class T>
    mps_status alloc(T *&ptr, size_t count) {
        size_t nbytes = sizeof(T) * (count > 0 ? count : 1);
        if (limit && bytes + nbytes > limit)
            return fail(MPS_E_OUT_OF_MEMORY, "allocation of %zu bytes exceeds the test limit",
                        nbytes);
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, nbytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MPS_E_OUT_OF_MEMORY, "hipMalloc(%zu): %s", nbytes, hipGetErrorString(e));
        }
        allocs.push_back(p);
        bytes += nbytes;
        ptr = (T *)p;
        return MPS_OK;
    }
    void release() {
        for (void *p : allocs) hipFree(p);
        allocs.clear();
    }
};

extern "C" {

const char *mps_last_error(void) { return g_err.c_str(); }

int32_t mps_version(void) { return 100; }

mps_status mps_device_count(int32_t *n) {
    if (!n) return fail(MPS_E_INVALID_ARG, "n is NULL");
    int c = 0;
    hipError_t e = hipGetDeviceCount(&c);
    if (e != hipSuccess || c <= 0) {
        (void)hipGetLastError();
        *n = 0;
        return fail(MPS_E_DEVICE, "no GPU visible (%s)",
                    e != hipSuccess ? hipGetErrorString(e) : "0 devices");
    }
    *n = c;
    return MPS_OK;
}

static mps_status check_params(const mps_params *p) {
    if (!p) return fail(MPS_E_INVALID_ARG, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(MPS_E_INVALID_ARG, "grid dimensions must be >= 1 (got %d x %d x %d)", p->nx,
                    p->ny, p->nz);
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    if (N > (int64_t)INT32_MAX / 128)
        return fail(MPS_E_INVALID_ARG, "too many blocks (%lld)", (long long)N);
    if (p->n_scen < 1 || p->n_scen > MPS_MAX_SCENARIOS)
        return fail(MPS_E_INVALID_ARG, "n_scen must be in 1..%d (got %d)", MPS_MAX_SCENARIOS,
                    p->n_scen);
    if (p->n_periods < 1 || p->n_periods > MPS_MAX_PERIODS)
        return fail(MPS_E_INVALID_ARG, "n_periods must be in 1..%d (got %d)", MPS_MAX_PERIODS,
                    p->n_periods);
    if (p->precedence != MPS_PREC_GRID_1_5 && p->precedence != MPS_PREC_CSR)
        return fail(MPS_E_INVALID_ARG, "precedence must be MPS_PREC_GRID_1_5 or MPS_PREC_CSR (got %d)",
                    p->precedence);
    if (!isfinite(p->discount_rate) || p->discount_rate <= -1.0)
        return fail(MPS_E_INVALID_ARG, "discount_rate must be finite and > -1");
    if (!isfinite(p->lambda)) return fail(MPS_E_INVALID_ARG, "lambda must be finite");
    if (!isfinite(p->pen_proc) || p->pen_proc < 0 || !isfinite(p->pen_mine) || p->pen_mine < 0)
        return fail(MPS_E_INVALID_ARG, "penalties must be finite and >= 0");
    if (!isfinite(p->proc_cap) || !isfinite(p->mine_cap))
        return fail(MPS_E_INVALID_ARG, "capacities must be finite");
    return MPS_OK;
}

// Explicit predecessor lists: validated, and their transpose (successor
// lists, each in increasing block index) built on the host.
static mps_status check_lists(int64_t N, const int32_t *pred_ptr, const int32_t *pred_idx,
                              std::vector<int32_t> &sp, std::vector<int32_t> &si) {
    if (!pred_ptr || !pred_idx)
        return fail(MPS_E_INVALID_ARG, "MPS_PREC_CSR needs pred_ptr and pred_idx");
    if (pred_ptr[0] != 0) return fail(MPS_E_INVALID_ARG, "pred_ptr[0] must be 0");
    for (int64_t b = 0; b < N; ++b) {
        const int64_t deg = (int64_t)pred_ptr[b + 1] - pred_ptr[b];
        if (deg < 0 || deg > MPS_MAX_DEGREE)
            return fail(MPS_E_INVALID_ARG, "block %lld has %lld predecessors (0..%d allowed)",
                        (long long)b, (long long)deg, MPS_MAX_DEGREE);
        for (int32_t j = pred_ptr[b]; j < pred_ptr[b + 1]; ++j) {
            const int32_t a = pred_idx[j];
            if (a < 0 || a >= N || a == b)
                return fail(MPS_E_INVALID_ARG, "block %lld: predecessor %d is out of range or "
                            "the block itself", (long long)b, a);
            for (int32_t i = pred_ptr[b]; i < j; ++i)
                if (pred_idx[i] == a)
                    return fail(MPS_E_INVALID_ARG, "block %lld lists predecessor %d twice",
                                (long long)b, a);
        }
    }
    const int64_t nnz = pred_ptr[N];
    sp.assign((size_t)N + 1, 0);
    si.assign((size_t)(nnz > 0 ? nnz : 1), 0);
    for (int64_t c = 0; c < N; ++c)
        for (int32_t j = pred_ptr[c]; j < pred_ptr[c + 1]; ++j) ++sp[(size_t)pred_idx[j] + 1];
    for (int64_t b = 0; b < N; ++b) {
        if (sp[b + 1] > MPS_MAX_DEGREE)
            return fail(MPS_E_INVALID_ARG, "block %lld has %d successors (0..%d allowed)",
                        (long long)b, sp[b + 1], MPS_MAX_DEGREE);
        sp[b + 1] += sp[b];
    }
    std::vector<int32_t> fill(sp.begin(), sp.end() - 1);
    for (int64_t c = 0; c < N; ++c)
        for (int32_t j = pred_ptr[c]; j < pred_ptr[c + 1]; ++j)
            si[(size_t)fill[pred_idx[j]]++] = (int32_t)c;
    return MPS_OK;
}

mps_status mps_build_model(const mps_params *prm, const float *v, const uint32_t *ore_bits,
                           const double *ton, const int32_t *pred_ptr, const int32_t *pred_idx,
                           void *stream, mps_model **out) {
    if (!out) return fail(MPS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mps_status st = check_params(prm);
    if (st != MPS_OK) return st;
    std::vector<int32_t> succ_ptr, succ_idx;
    if (prm->precedence == MPS_PREC_CSR) {
        const int64_t Nl = (int64_t)prm->nx * prm->ny * prm->nz;
        if ((st = check_lists(Nl, pred_ptr, pred_idx, succ_ptr, succ_idx)) != MPS_OK) return st;
    } else if (pred_ptr || pred_idx) {
        return fail(MPS_E_INVALID_ARG, "predecessor lists are given only with MPS_PREC_CSR");
    }
    if (!v || !ore_bits || !ton) return fail(MPS_E_INVALID_ARG, "v, ore_bits and ton are required");
    int32_t ndev = 0;
    if ((st = mps_device_count(&ndev)) != MPS_OK) return st;
    if (!is_device_ptr(v) || !is_device_ptr(ore_bits) || !is_device_ptr(ton))
        return fail(MPS_E_INVALID_ARG, "v, ore_bits and ton must be device pointers");
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_build_model during capture");

    mps_model *m = new mps_model();
    hipGetDevice(&m->device);
    m->prm = *prm;
    if (const char *lim = getenv("MPS_TEST_ALLOC_LIMIT")) m->limit = (size_t)strtoull(lim, 0, 10);
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device) ==
            hipSuccess &&
        lds > 0)
        m->max_lds = lds;

    DevModel &d = m->d;
    d.nx = prm->nx;
    d.ny = prm->ny;
    d.nz = prm->nz;
    d.N = (int64_t)prm->nx * prm->ny * prm->nz;
    d.S = prm->n_scen;
    d.T = prm->n_periods;
    d.W = (d.S + 31) / 32;
    d.lambda = prm->lambda;
    d.pen_proc = prm->pen_proc;
    d.pen_mine = prm->pen_mine;
    d.pcap = prm->proc_cap;
    d.mcap = prm->mine_cap;
    const int64_t N = d.N;
    const int32_t S = d.S, T = d.T, W = d.W;

    // tonnages: validated and summarised on the host
    std::vector<double> th((size_t)N);
    hipError_t e = hipMemcpy(th.data(), ton, sizeof(double) * N, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        delete m;
        return dev_fail(e, "copy of ton");
    }
    double tmin = INFINITY, tmax = 0.0;
    for (int64_t b = 0; b < N; ++b) {
        if (!(th[b] > 0.0) || !isfinite(th[b])) {
            delete m;
            return fail(MPS_E_INVALID_ARG, "ton[%lld] = %g must be finite and > 0", (long long)b,
                        th[b]);
        }
        tmin = fmin(tmin, th[b]);
        tmax = fmax(tmax, th[b]);
    }
    d.ton_min = tmin;
    d.ton_max = tmax;

    float *v_, *ton32, *mb32, *Vb32, *e32;
    uint32_t *ore_, *full_add, *full_rem;
    double *ton64, *mb64, *Vb64, *Ns, *O, *M, *d64;
    int8_t *p;
    int32_t *trng;
    AddEntry *padd;
    RemEntry *prem;
    DevScalars *sc;
#define ALLOC(ptr, cnt)                      \
    if ((st = m->alloc(ptr, cnt)) != MPS_OK) { \
        m->release();                        \
        delete m;                            \
        return st;                           \
    }
    const int64_t vld = (N + 31) / 32 * 32;   // 128-byte rows
    ALLOC(v_, (size_t)S * vld);
    ALLOC(ore_, (size_t)W * N);
    ALLOC(ton64, N);
    ALLOC(ton32, N);
    ALLOC(mb64, N);
    ALLOC(Vb64, N);
    ALLOC(mb32, N);
    ALLOC(Vb32, N);
    ALLOC(d64, T + 1);
    // Mutable search state (schedule, per-scenario NPV, period tonnages,
    // scalars, penalty tables) in one arena, so that saving or restoring it
    // is one device copy.
    {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off = (off + bytes + 255) & ~(size_t)255;
            return o;
        };
        const size_t o_p = take((size_t)N), o_Ns = take(8 * (size_t)S),
                     o_O = take(8 * (size_t)T * S), o_M = take(8 * (size_t)T),
                     o_e = take(4 * ((size_t)S + 64)), o_sc = take(sizeof(DevScalars)),
                     o_fa = take(4 * (size_t)T * W), o_fr = take(4 * (size_t)T * W),
                     o_rg = take(16 * (size_t)T),
                     o_pa = take(sizeof(AddEntry) * (size_t)T * S),
                     o_pr = take(sizeof(RemEntry) * (size_t)T * S);
        char *arena = nullptr;
        ALLOC(arena, off);
        m->arena = arena;
        m->arena_bytes = off;
        p = (int8_t *)(arena + o_p);
        Ns = (double *)(arena + o_Ns);
        O = (double *)(arena + o_O);
        M = (double *)(arena + o_M);
        e32 = (float *)(arena + o_e);
        sc = (DevScalars *)(arena + o_sc);
        full_add = (uint32_t *)(arena + o_fa);
        full_rem = (uint32_t *)(arena + o_fr);
        trng = (int32_t *)(arena + o_rg);
        padd = (AddEntry *)(arena + o_pa);
        prem = (RemEntry *)(arena + o_pr);
    }
    ListRec *blk_rec = nullptr;
    ALLOC(blk_rec, N);
    uint32_t *tmark = nullptr;
    ALLOC(tmark, (size_t)(N + 63) / 64);
    ALLOC(m->partial, (size_t)m->chunks * (S + 1) * (T + 1));
    ALLOC(m->obj_dev, 8);
    {
        char *rw = nullptr;
        ALLOC(rw, relaxed_ws_bytes(d));
        m->relax_ws = rw;
        char *gw = nullptr;
        ALLOC(gw, repair_gather_bytes(S, W));
        m->gather = gw;
        ALLOC(m->rep_first, N);
        ALLOC(m->cmark, N);
    }
    if (prm->precedence == MPS_PREC_CSR) {
        const size_t nnz = (size_t)pred_ptr[N];
        int32_t *pp_ = nullptr, *pi_ = nullptr, *sp_ = nullptr, *si_ = nullptr;
        ALLOC(pp_, (size_t)N + 1);
        ALLOC(pi_, nnz);
        ALLOC(sp_, (size_t)N + 1);
        ALLOC(si_, nnz);
        hipError_t ce = hipMemcpy(pp_, pred_ptr, 4 * ((size_t)N + 1), hipMemcpyHostToDevice);
        if (ce == hipSuccess && nnz) ce = hipMemcpy(pi_, pred_idx, 4 * nnz, hipMemcpyHostToDevice);
        if (ce == hipSuccess)
            ce = hipMemcpy(sp_, succ_ptr.data(), 4 * ((size_t)N + 1), hipMemcpyHostToDevice);
        if (ce == hipSuccess && nnz)
            ce = hipMemcpy(si_, succ_idx.data(), 4 * nnz, hipMemcpyHostToDevice);
        if (ce != hipSuccess) {
            m->release();
            delete m;
            return dev_fail(ce, "copy of the predecessor lists");
        }
        d.csr = 1;
        d.pred_ptr = pp_;
        d.pred_idx = pi_;
        d.succ_ptr = sp_;
        d.succ_idx = si_;
    }
#undef ALLOC
    d.v = v_;
    d.vld = vld;
    d.ore = ore_;
    d.ton64 = ton64;
    d.ton32 = ton32;
    d.mb64 = mb64;
    d.Vb64 = Vb64;
    d.mb32 = mb32;
    d.Vb32 = Vb32;
    d.p = p;
    d.Ns = Ns;
    d.O = O;
    d.M = M;
    d.e32 = e32;
    d.sc = sc;
    d.d64 = d64;
    d.tab.full_add = full_add;
    d.tab.full_rem = full_rem;
    d.tab.rng = trng;
    d.tab.add_packed = padd;
    d.tab.rem_packed = prem;
    d.blk_rec = blk_rec;
    d.tmark = tmark;

    // discount factors: d(0) = 1, d(t) = d(t-1)/(1+rate), d(T) = 0
    std::vector<double> dh((size_t)T + 1);
    dh[0] = 1.0;
    for (int32_t t = 1; t < T; ++t) dh[t] = dh[t - 1] / (1.0 + prm->discount_rate);
    dh[T] = 0.0;
    std::vector<float> t32((size_t)N);
    for (int64_t b = 0; b < N; ++b) t32[b] = (float)th[b];

    auto chk = [&](hipError_t err, const char *what) -> mps_status {
        if (err == hipSuccess) return MPS_OK;
        m->release();
        delete m;
        return dev_fail(err, what);
    };
    if ((st = chk(hipMemsetAsync(v_, 0, sizeof(float) * S * vld, hs), "padding of v")) != MPS_OK)
        return st;
    if ((st = chk(hipMemcpy2DAsync(v_, sizeof(float) * vld, v, sizeof(float) * N,
                                   sizeof(float) * N, S, hipMemcpyDeviceToDevice, hs),
                  "copy of v")) != MPS_OK)
        return st;
    if ((st = chk(hipMemcpyAsync(ore_, ore_bits, sizeof(uint32_t) * W * N,
                                 hipMemcpyDeviceToDevice, hs),
                  "copy of ore_bits")) != MPS_OK)
        return st;
    if ((st = chk(hipMemcpyAsync(ton64, ton, sizeof(double) * N, hipMemcpyDeviceToDevice, hs),
                  "copy of ton")) != MPS_OK)
        return st;
    if ((st = chk(hipMemcpyAsync(ton32, t32.data(), sizeof(float) * N, hipMemcpyHostToDevice, hs),
                  "copy of ton32")) != MPS_OK)
        return st;
    if ((st = chk(hipMemsetD32Async((hipDeviceptr_t)m->rep_first, INT32_MAX, (size_t)N, hs),
                  "repair marks")) != MPS_OK)
        return st;
    if ((st = chk(hipMemsetAsync(tmark, 0, sizeof(uint32_t) * ((N + 63) / 64), hs),
                  "tile marks")) != MPS_OK)
        return st;
    if ((st = chk(hipMemcpyAsync(d64, dh.data(), sizeof(double) * (T + 1),
                                 hipMemcpyHostToDevice, hs),
                  "copy of discount table")) != MPS_OK)
        return st;
    if ((st = chk(launch_block_stats(d, mb32, Vb32, mb64, Vb64, hs), "block statistics")) !=
        MPS_OK)
        return st;
    if ((st = chk(launch_relaxed_init(d, m->relax_ws, hs), "relaxed stencil")) != MPS_OK)
        return st;
    // initial schedule: everything in period 0
    std::vector<int8_t> zero((size_t)N, 0);
    if ((st = chk(hipMemcpyAsync(p, zero.data(), N, hipMemcpyHostToDevice, hs), "schedule")) !=
        MPS_OK)
        return st;
    if ((st = chk(launch_set_schedule(d, p, m->partial, m->chunks, hs), "set schedule")) != MPS_OK)
        return st;
    if ((st = chk(hipStreamSynchronize(hs), "build synchronise")) != MPS_OK) return st;
    *out = m;
    return MPS_OK;
}

mps_status mps_destroy_model(mps_model *m) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    DeviceGuard g(m->device);
    hipDeviceSynchronize();
    m->release();
    delete m;
    return MPS_OK;
}

mps_status mps_model_dims(const mps_model *m, int64_t *N, int32_t *S, int32_t *T) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (N) *N = m->d.N;
    if (S) *S = m->d.S;
    if (T) *T = m->d.T;
    return MPS_OK;
}

mps_status mps_set_schedule(mps_model *m, const int8_t *p, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (!p) return fail(MPS_E_INVALID_ARG, "p is NULL");
    DeviceGuard g(m->device);
    hipError_t e = launch_set_schedule(m->d, p, m->partial, m->chunks, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "set schedule");
}

mps_status mps_get_schedule(mps_model *m, int8_t *p, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (!p) return fail(MPS_E_INVALID_ARG, "p is NULL");
    DeviceGuard g(m->device);
    hipError_t e = hipMemcpyAsync(p, m->d.p, m->d.N, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "copy of schedule");
}

mps_status mps_objective_async(mps_model *m, double *out, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (!out) return fail(MPS_E_INVALID_ARG, "out is NULL");
    DeviceGuard g(m->device);
    hipError_t e = launch_objective_copy(m->d, out, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "objective");
}

mps_status mps_get_objective(mps_model *m, mps_objective *out, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (!out) return fail(MPS_E_INVALID_ARG, "out is NULL");
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_get_objective during capture");
    DeviceGuard g(m->device);
    hipError_t e = launch_objective_copy(m->d, m->obj_dev, hs);
    double h[7];
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, m->obj_dev, sizeof(h), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return dev_fail(e, "objective");
    out->mu = h[0];
    out->sigma = h[1];
    out->R = h[2];
    out->Pp = h[3];
    out->Pm = h[4];
    out->J = h[5];
    out->n_prec_viol = (int64_t)h[6];
    return MPS_OK;
}

static mps_status check_moves(const mps_model *m, const mps_moves *mv) {
    if (!mv) return fail(MPS_E_INVALID_ARG, "moves is NULL");
    if (mv->exhaustive) {
        int32_t D = mv->include_never ? m->d.T + 1 : m->d.T;
        if (m->d.N * (int64_t)D >= ((int64_t)1 << 31))
            return fail(MPS_E_INVALID_ARG, "N*D = %lld moves exceed 2^31 - 1",
                        (long long)(m->d.N * D));
        return MPS_OK;
    }
    if (mv->n < 0 || mv->n >= ((int64_t)1 << 31))
        return fail(MPS_E_INVALID_ARG, "moves->n = %lld out of range", (long long)mv->n);
    if (mv->n > 0 && (!mv->block || !mv->period))
        return fail(MPS_E_INVALID_ARG, "list moves need block and period arrays");
    return MPS_OK;
}

// The evaluation kernels keep one tile's tables in LDS: S and T together must
// leave them room.
// Calls whose arithmetic is the base objective's refuse a model with an
// objective variant.
static mps_status no_variant(const mps_model *m, const char *what) {
    if (has_variant(m->d))
        return fail(MPS_E_INVALID_ARG,
                    "%s uses the base objective (std risk, no value multiplier); this model "
                    "has an objective variant set", what);
    return MPS_OK;
}

static mps_status check_eval_lds(const mps_model *m, const mps_moves &mv) {
    if (has_variant(m->d)) {
        if (m->d.S > kVariantMaxScen)
            return fail(MPS_E_INVALID_ARG,
                        "evaluation under an objective variant supports S <= %d (got %d)",
                        kVariantMaxScen, m->d.S);
        const size_t need = eval_var_lds_bytes(m->d);
        if (need > (size_t)m->max_lds)
            return fail(MPS_E_INVALID_ARG,
                        "evaluation under an objective variant keeps 8*T*S + 4*S*(T+1) bytes "
                        "of tables in LDS (%zu), device allows %d", need, m->max_lds);
        return MPS_OK;
    }
    const size_t need = eval_lds_bytes(m->d, mv);
    if (need > (size_t)m->max_lds)
        return fail(MPS_E_INVALID_ARG,
                    "evaluating moves of this model needs %zu bytes of LDS (T = %d periods of "
                    "%d ore words per tile), device allows %d: reduce S or T",
                    need, m->d.T, m->d.W, m->max_lds);
    return MPS_OK;
}

mps_status mps_eval_moves(mps_model *m, const mps_moves *moves, float *score, uint8_t *flags,
                          float *d_risk, float *d_pen_proc, float *d_pen_mine, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    mps_status st = check_moves(m, moves);
    if (st != MPS_OK) return st;
    const int64_t n_moves =
        moves->exhaustive ? m->d.N * (int64_t)(moves->include_never ? m->d.T + 1 : m->d.T)
                          : moves->n;
    if (n_moves == 0) return MPS_OK;
    if (!score || !flags) return fail(MPS_E_INVALID_ARG, "score and flags are required");
    if ((st = check_eval_lds(m, *moves)) != MPS_OK) return st;
    int nc = (d_risk != nullptr) + (d_pen_proc != nullptr) + (d_pen_mine != nullptr);
    if (nc != 0 && nc != 3)
        return fail(MPS_E_INVALID_ARG, "component outputs must be all given or all NULL");
    DeviceGuard g(m->device);
    hipError_t e = launch_eval(m->d, *moves, score, flags, d_risk, d_pen_proc, d_pen_mine,
                               (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "eval moves");
}

size_t mps_topk_ws_bytes(int64_t n, int32_t k) {
    if (k < 1) k = 1;
    return topk_ws_bytes(n, k);
}

mps_status mps_topk(const float *score, const uint8_t *flags, int64_t n, int32_t k,
                    uint8_t require, uint8_t forbid, int64_t *idx, float *top_score,
                    int32_t *count, void *ws, size_t ws_bytes, void *stream) {
    if (k < 1 || k > MPS_MAX_TOPK)
        return fail(MPS_E_INVALID_ARG, "k must be in 1..%d (got %d)", MPS_MAX_TOPK, k);
    if (n < 0 || n >= ((int64_t)1 << 31))
        return fail(MPS_E_INVALID_ARG, "n = %lld out of range", (long long)n);
    if ((n > 0 && (!score || !flags)) || !idx || !count || !ws)
        return fail(MPS_E_INVALID_ARG, "score, flags, idx, count and ws are required");
    if (ws_bytes < topk_ws_bytes(n, k))
        return fail(MPS_E_INVALID_ARG, "workspace of %zu bytes is below the %zu needed", ws_bytes,
                    topk_ws_bytes(n, k));
    hipError_t e = launch_topk(score, flags, n, k, require, forbid, idx, top_score, count, ws,
                               (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "topk");
}

mps_status mps_repair(mps_model *m, const mps_moves *moves, const int64_t *idx,
                      const int32_t *count, int32_t max_cand, int32_t hard_capacity,
                      int32_t *applied, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    mps_status st = check_moves(m, moves);
    if (st != MPS_OK) return st;
    if ((st = no_variant(m, "mps_repair")) != MPS_OK) return st;
    if (!idx || !count) return fail(MPS_E_INVALID_ARG, "idx and count are required");
    if (max_cand < 0 || max_cand > MPS_MAX_TOPK)
        return fail(MPS_E_INVALID_ARG, "max_cand must be in 0..%d", MPS_MAX_TOPK);
    if (m->d.S > kRepairMaxScen)
        return fail(MPS_E_INVALID_ARG, "repair supports S <= %d (got %d)", kRepairMaxScen,
                    m->d.S);
    size_t need = repair_lds_bytes(m->d, max_cand);
    if (need > (size_t)m->max_lds)
        return fail(MPS_E_INVALID_ARG,
                    "repair state needs %zu bytes of LDS (O rows, period map, two record "
                    "batches), device allows %d", need, m->max_lds);
    DeviceGuard g(m->device);
    hipError_t e = launch_repair(m->d, *moves, idx, count, max_cand, hard_capacity, applied,
                                 m->gather, m->rep_first, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "repair");
}

mps_status mps_repair_cascade(mps_model *m, const mps_moves *moves, const int64_t *idx,
                              const int32_t *count, int32_t max_cand, int32_t hard_capacity,
                              int32_t max_set, int32_t *applied, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    mps_status st = check_moves(m, moves);
    if (st != MPS_OK) return st;
    if ((st = no_variant(m, "mps_repair_cascade")) != MPS_OK) return st;
    if (!idx || !count) return fail(MPS_E_INVALID_ARG, "idx and count are required");
    if (max_cand < 0 || max_cand > MPS_MAX_TOPK)
        return fail(MPS_E_INVALID_ARG, "max_cand must be in 0..%d", MPS_MAX_TOPK);
    if (max_set < 1 || max_set > kCascadeMaxSet)
        return fail(MPS_E_INVALID_ARG, "max_set must be in 1..%d (got %d)", kCascadeMaxSet,
                    max_set);
    const size_t need = cascade_lds_bytes(m->d);
    if (need > (size_t)m->max_lds)
        return fail(MPS_E_INVALID_ARG,
                    "cascading repair keeps 8*(T*S + 2S + 2T + 1) bytes of state in LDS "
                    "(%zu with its set lists); the device allows %d", need, m->max_lds);
    DeviceGuard g(m->device);
    hipError_t e = launch_cascade(m->d, *moves, idx, count, max_cand, hard_capacity, max_set,
                                  applied, m->cmark, m->partial, m->chunks, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "cascading repair");
}

size_t mps_state_bytes(const mps_model *m) { return m ? m->arena_bytes : 0; }

mps_status mps_state_save(mps_model *m, void *buf, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (!buf) return fail(MPS_E_INVALID_ARG, "buf is NULL");
    DeviceGuard g(m->device);
    hipError_t e = hipMemcpyAsync(buf, m->arena, m->arena_bytes, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "state save");
}

mps_status mps_state_restore(mps_model *m, const void *buf, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (!buf) return fail(MPS_E_INVALID_ARG, "buf is NULL");
    DeviceGuard g(m->device);
    hipError_t e = hipMemcpyAsync(m->arena, buf, m->arena_bytes, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "state restore");
}

size_t mps_relaxed_saved_bytes(const mps_model *m) {
    return m ? relaxed_saved_bytes(m->d) : 0;
}

static mps_status check_relax(const mps_relax_params *rp) {
    if (!rp) return fail(MPS_E_INVALID_ARG, "relax params are NULL");
    if (!isfinite(rp->mu_proc) || !isfinite(rp->mu_mine) || !isfinite(rp->mu_prec) ||
        rp->mu_proc < 0 || rp->mu_mine < 0 || rp->mu_prec < 0)
        return fail(MPS_E_INVALID_ARG, "relaxed penalty weights must be finite and >= 0");
    return MPS_OK;
}

mps_status mps_relaxed_fwd(mps_model *m, const float *x, const mps_relax_params *rp,
                           double *J_out, void *saved, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    mps_status st = check_relax(rp);
    if (st != MPS_OK) return st;
    if ((st = no_variant(m, "mps_relaxed_fwd")) != MPS_OK) return st;
    if (!x || !saved) return fail(MPS_E_INVALID_ARG, "x and saved are required");
    DeviceGuard g(m->device);
    hipError_t e = launch_relaxed_fwd(m->d, x, *rp, J_out, saved, m->relax_ws, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "relaxed forward");
}

mps_status mps_relaxed_bwd(mps_model *m, const float *x, const mps_relax_params *rp,
                           const void *saved, const double *dJ, float *grad_x, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    mps_status st = check_relax(rp);
    if (st != MPS_OK) return st;
    if ((st = no_variant(m, "mps_relaxed_bwd")) != MPS_OK) return st;
    if (!x || !saved || !grad_x) return fail(MPS_E_INVALID_ARG, "x, saved and grad_x are required");
    DeviceGuard g(m->device);
    hipError_t e = launch_relaxed_bwd(m->d, x, *rp, saved, dJ, grad_x, m->relax_ws, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "relaxed backward");
}

size_t mps_rank_ws_bytes(const mps_model *m, int32_t k) {
    if (!m) return 0;
    if (k < 1) k = 1;
    return rank_ws_bytes(m->d, k);
}

mps_status mps_rank_moves(mps_model *m, const float *grad_x, int32_t k, int32_t *block,
                          int8_t *period, float *gain, int32_t *count, void *ws,
                          size_t ws_bytes, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (k < 1 || k > MPS_MAX_TOPK)
        return fail(MPS_E_INVALID_ARG, "k must be in 1..%d (got %d)", MPS_MAX_TOPK, k);
    if (!grad_x || !block || !period || !count || !ws)
        return fail(MPS_E_INVALID_ARG, "grad_x, block, period, count and ws are required");
    {
        const mps_status vs = no_variant(m, "mps_rank_moves");
        if (vs != MPS_OK) return vs;
    }
    if (m->d.N * (int64_t)(m->d.T + 1) >= ((int64_t)1 << 31))
        return fail(MPS_E_INVALID_ARG, "too many moves to rank");
    if (ws_bytes < rank_ws_bytes(m->d, k))
        return fail(MPS_E_INVALID_ARG, "workspace of %zu bytes is below the %zu needed", ws_bytes,
                    rank_ws_bytes(m->d, k));
    DeviceGuard g(m->device);
    hipError_t e = launch_rank(m->d, grad_x, k, block, period, gain, count, ws, (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "rank moves");
}

mps_status mps_set_objective_variant(mps_model *m, const double *mult, int32_t risk,
                                     double cvar_alpha, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (risk != MPS_RISK_STD && risk != MPS_RISK_CVAR)
        return fail(MPS_E_INVALID_ARG, "risk must be MPS_RISK_STD or MPS_RISK_CVAR (got %d)", risk);
    if (risk == MPS_RISK_CVAR && !(cvar_alpha > 0.0 && cvar_alpha <= 1.0))
        return fail(MPS_E_INVALID_ARG, "cvar_alpha must be in (0, 1] (got %g)", cvar_alpha);
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_set_objective_variant during capture");
    DevModel &d = m->d;
    const int32_t S = d.S, T = d.T, T1 = d.T + 1;
    if (mult) {
        for (int64_t i = 0; i < (int64_t)S * T; ++i)
            if (!isfinite(mult[i]))
                return fail(MPS_E_INVALID_ARG, "mult[%lld] = %g is not finite", (long long)i,
                            mult[i]);
    }
    DeviceGuard g(m->device);
    mps_status st;
    if (mult && !m->wmult) {
        double *w64 = nullptr;
        float *w32 = nullptr;
        if ((st = m->alloc(w64, (size_t)S * T1)) != MPS_OK) return st;
        if ((st = m->alloc(w32, (size_t)S * T1)) != MPS_OK) return st;
        m->wmult = w64;
        m->wmult32 = w32;
    }
    hipError_t e = hipSuccess;
    if (mult) {
        // w[s][t] = d(t) sigma(s,t) in FP64 on the host, d(T) = 0
        std::vector<double> dh(T1), w(S * (size_t)T1);
        std::vector<float> w32(S * (size_t)T1);
        e = hipMemcpy(dh.data(), d.d64, sizeof(double) * T1, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return dev_fail(e, "discount table");
        for (int32_t s = 0; s < S; ++s)
            for (int32_t t = 0; t < T1; ++t) {
                const double x = t < T ? dh[t] * mult[(size_t)s * T + t] : 0.0;
                w[(size_t)s * T1 + t] = x;
                w32[(size_t)s * T1 + t] = (float)x;
            }
        e = hipMemcpyAsync(m->wmult, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m->wmult32, w32.data(), sizeof(float) * w32.size(),
                               hipMemcpyHostToDevice, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) return dev_fail(e, "multiplier table");
    }
    d.wmult = mult ? m->wmult : nullptr;
    d.wmult32 = mult ? m->wmult32 : nullptr;
    d.risk = risk;
    d.alpha = risk == MPS_RISK_CVAR ? cvar_alpha : 0.0;
    // the state of the current schedule under the new objective
    e = launch_set_schedule(d, d.p, m->partial, m->chunks, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "objective variant");
}

mps_status mps_lns_sa(mps_model *m, const mps_lns_params *prm, const double *u, double *traj,
                      mps_lns_stats *out, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    if (!prm || !u) return fail(MPS_E_INVALID_ARG, "params and u are required");
    {
        const mps_status vs = no_variant(m, "mps_lns_sa");
        if (vs != MPS_OK) return vs;
    }
    const mps_lns_params P = *prm;
    if (P.n_iter < 0 || P.tile < 1 || P.k < 1 || P.k > MPS_MAX_TOPK || P.max_rounds < 0)
        return fail(MPS_E_INVALID_ARG,
                    "need n_iter >= 0, tile >= 1, 1 <= k <= %d, max_rounds >= 0", MPS_MAX_TOPK);
    if (!isfinite(P.eps_max) || !isfinite(P.temp0) || !isfinite(P.cool) || P.eps_max < 0 ||
        P.temp0 < 0 || P.cool < 0)
        return fail(MPS_E_INVALID_ARG, "eps_max, temp0 and cool must be finite and >= 0");
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_lns_sa during capture");
    const DevModel &d = m->d;
    if (d.N * (int64_t)d.T >= ((int64_t)1 << 31)) return fail(MPS_E_INVALID_ARG, "too many moves");
    if (d.S > kRepairMaxScen)
        return fail(MPS_E_INVALID_ARG, "repair supports S <= %d (got %d)", kRepairMaxScen, d.S);
    if (repair_lds_bytes(d, P.k) > (size_t)m->max_lds)
        return fail(MPS_E_INVALID_ARG, "repair state does not fit in LDS");
    mps_status st;
    {
        mps_moves lst{};
        if ((st = check_eval_lds(m, lst)) != MPS_OK) return st;
    }
    const int32_t kx = (d.nx + P.tile - 1) / P.tile, ky = (d.ny + P.tile - 1) / P.tile;
    const int32_t K = kx * ky;
    DeviceGuard g(m->device);
    SearchBufs B;
    const int64_t nm = d.N * (int64_t)d.T;
    char *cur = B.get<char>(m->arena_bytes), *best = B.get<char>(m->arena_bytes);
    uint8_t *reg = B.get<uint8_t>(d.N);
    int32_t *lb = B.get<int32_t>(nm);
    int8_t *lt = B.get<int8_t>(nm);
    float *score = B.get<float>(nm);
    uint8_t *flags = B.get<uint8_t>(nm);
    char *tws = B.get_zeroed(topk_ws_bytes(nm, P.k), topk_ws_zero_bytes(), hs);
    int64_t *idx = B.get<int64_t>(P.k);
    int32_t *cnt = B.get<int32_t>(4);   // [0] list length, [1] top-k count, [2] applied
    double *objd = B.get<double>(8);
    if (!cur || !best || !reg || !lb || !lt || !score || !flags || !tws || !idx || !cnt || !objd)
        return fail(MPS_E_OUT_OF_MEMORY, "LNS buffers");
    hipError_t e = hipSuccess;
    auto objective = [&](double o[7]) {
        if (e == hipSuccess) e = launch_objective_copy(d, objd, hs);
        if (e == hipSuccess) e = hipMemcpyAsync(o, objd, 7 * sizeof(double), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
    };
    auto read_int = [&](const int32_t *src, int32_t &v) {
        if (e == hipSuccess) e = hipMemcpyAsync(&v, src, sizeof(int32_t), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
    };
    e = hipMemcpyAsync(cur, m->arena, m->arena_bytes, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(best, m->arena, m->arena_bytes, hipMemcpyDeviceToDevice, hs);
    double o[7];
    objective(o);
    double J_best = o[5], R_cur = o[2], P_cur = o[3] + o[4];
    int64_t steps = 0, n_acc = 0, n_eval = 0, n_app = 0;
    for (int32_t it = 0; it < P.n_iter && e == hipSuccess; ++it) {
        const double eps = P.eps_max * (1.0 - (double)it / P.n_iter);
        double temp = P.temp0;
        for (int32_t j = 0; j < it; ++j) temp *= P.cool;
        for (int32_t i = 0; i < K && e == hipSuccess; ++i) {
            // the current schedule, its tile destroyed, the state re-derived
            e = hipMemcpyAsync(m->arena, cur, m->arena_bytes, hipMemcpyDeviceToDevice, hs);
            const int32_t tx = i % kx, ty = i / kx;
            if (e == hipSuccess)
                e = launch_lns_destroy(d, tx * P.tile, std::min(d.nx, (tx + 1) * P.tile),
                                       ty * P.tile, std::min(d.ny, (ty + 1) * P.tile), reg, lb,
                                       lt, cnt, hs);
            if (e == hipSuccess) e = launch_set_schedule(d, d.p, m->partial, m->chunks, hs);
            int32_t nl = 0;
            read_int(cnt, nl);
            mps_moves lst{};
            lst.exhaustive = 0;
            lst.include_never = 1;
            lst.n = nl;
            lst.block = lb;
            lst.period = lt;
            for (int32_t r = 0; r < P.max_rounds && e == hipSuccess && nl > 0; ++r) {
                e = launch_eval(d, lst, score, flags, nullptr, nullptr, nullptr, hs);
                if (e == hipSuccess)
                    e = launch_topk(score, flags, nl, P.k, MPS_PREC_OK, MPS_NOOP | MPS_BAD, idx,
                                    nullptr, cnt + 1, tws, hs);
                if (e == hipSuccess)
                    e = launch_repair(d, lst, idx, cnt + 1, P.k, 0, cnt + 2, m->gather,
                                      m->rep_first, hs);
                n_eval += nl;
                int32_t a = 0;
                read_int(cnt + 2, a);
                n_app += a;
                if (a == 0) break;
            }
            objective(o);
            if (e != hipSuccess) break;
            const double Pc = o[3] + o[4];
            const double f_cand = o[2] - (Pc - eps > 0.0 ? Pc - eps : 0.0);
            const double f_cur = R_cur - (P_cur - eps > 0.0 ? P_cur - eps : 0.0);
            const bool accept = f_cand > f_cur - u[(int64_t)it * K + i] * temp;
            if (traj) {
                traj[steps * 4 + 0] = o[5];
                traj[steps * 4 + 1] = o[2];
                traj[steps * 4 + 2] = Pc;
                traj[steps * 4 + 3] = accept ? 1.0 : 0.0;
            }
            ++steps;
            if (accept) {
                e = hipMemcpyAsync(cur, m->arena, m->arena_bytes, hipMemcpyDeviceToDevice, hs);
                R_cur = o[2];
                P_cur = Pc;
                ++n_acc;
                if (o[5] > J_best && e == hipSuccess) {
                    J_best = o[5];
                    e = hipMemcpyAsync(best, m->arena, m->arena_bytes, hipMemcpyDeviceToDevice, hs);
                }
            }
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(m->arena, best, m->arena_bytes, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return dev_fail(e, "LNS driver");
    if (out) {
        out->steps = steps;
        out->accepted = n_acc;
        out->evaluations = n_eval;
        out->applied = n_app;
        out->J_best = J_best;
    }
    return MPS_OK;
}

mps_status mps_greedy_init(mps_model *m, int32_t max_pass, int32_t *passes, int64_t *placed,
                           void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    {
        const mps_status vs = no_variant(m, "mps_greedy_init");
        if (vs != MPS_OK) return vs;
    }
    if (max_pass < 1) return fail(MPS_E_INVALID_ARG, "max_pass must be >= 1 (got %d)", max_pass);
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_greedy_init during capture");
    const DevModel &d = m->d;
    if (d.N >= ((int64_t)1 << 31)) return fail(MPS_E_INVALID_ARG, "too many blocks");
    const size_t lds = greedy_lds_bytes(d);
    if (lds > (size_t)m->max_lds)
        return fail(MPS_E_INVALID_ARG,
                    "greedy initializer keeps T*S = %lld tonnages in LDS (%zu bytes); the device "
                    "allows %d",
                    (long long)d.T * d.S, lds, m->max_lds);
    DeviceGuard g(m->device);
    SearchBufs B;
    char *ws = B.get<char>(greedy_ws_bytes(d));
    int8_t *p = B.get<int8_t>(d.N);
    int32_t *out = B.get<int32_t>(2);
    if (!ws || !p || !out) return fail(MPS_E_OUT_OF_MEMORY, "greedy initializer buffers");
    hipError_t e = launch_greedy(d, p, max_pass, ws, out, hs);
    if (e == hipSuccess) e = launch_set_schedule(d, p, m->partial, m->chunks, hs);
    int32_t h[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return dev_fail(e, "greedy initializer");
    if (passes) *passes = h[0];
    if (placed) *placed = h[1];
    return MPS_OK;
}

mps_status mps_search(mps_model *m, int32_t mode, int32_t k, const mps_relax_params *rp,
                      int32_t max_iter, mps_search_stats *out, void *stream) {
    if (!m) return fail(MPS_E_INVALID_ARG, "model is NULL");
    {
        const mps_status vs = no_variant(m, "mps_search");
        if (vs != MPS_OK) return vs;
    }
    if (mode != 0 && mode != 1) return fail(MPS_E_INVALID_ARG, "mode must be 0 or 1");
    if (k < 1 || k > MPS_MAX_TOPK)
        return fail(MPS_E_INVALID_ARG, "k must be in 1..%d (got %d)", MPS_MAX_TOPK, k);
    if (max_iter < 0) return fail(MPS_E_INVALID_ARG, "max_iter must be >= 0");
    mps_status st;
    if (mode == 1 && (st = check_relax(rp)) != MPS_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_search during capture");
    const DevModel &d = m->d;
    const int32_t D = d.T + 1;
    const int64_t nm = d.N * D;
    if (nm >= ((int64_t)1 << 31)) return fail(MPS_E_INVALID_ARG, "too many moves");
    if (d.S > kRepairMaxScen)
        return fail(MPS_E_INVALID_ARG, "repair supports S <= %d (got %d)", kRepairMaxScen, d.S);
    if (repair_lds_bytes(d, k) > (size_t)m->max_lds)
        return fail(MPS_E_INVALID_ARG, "repair state does not fit in LDS");
    {
        mps_moves all{};
        all.exhaustive = 1;
        all.include_never = 1;
        if ((st = check_eval_lds(m, all)) != MPS_OK) return st;
    }
    DeviceGuard g(m->device);
    SearchBufs B;
    float *score = B.get<float>(nm);
    uint8_t *flags = B.get<uint8_t>(nm);
    char *tws = B.get_zeroed(topk_ws_bytes(nm, k), topk_ws_zero_bytes(), hs);
    int64_t *idx = B.get<int64_t>(k);
    int32_t *cnt = B.get<int32_t>(4);
    float *x = nullptr, *grad = nullptr, *gain = nullptr, *lscore = nullptr;
    char *saved = nullptr, *rws = nullptr, *ltws = nullptr;
    int32_t *rblk = nullptr;
    int8_t *rper = nullptr;
    uint8_t *lflags = nullptr;
    if (mode == 1) {
        x = B.get<float>((size_t)d.N * d.T);
        grad = B.get<float>((size_t)d.N * d.T);
        saved = B.get<char>(relaxed_saved_bytes(d));
        rws = B.get_zeroed(rank_ws_bytes(d, k), rank_ws_bytes(d, k), hs);
        rblk = B.get<int32_t>(k);
        rper = B.get<int8_t>(k);
        gain = B.get<float>(k);
        lscore = B.get<float>(k);
        lflags = B.get<uint8_t>(k);
        ltws = B.get_zeroed(topk_ws_bytes(k, k), topk_ws_zero_bytes(), hs);
    }
    if (!score || !flags || !tws || !idx || !cnt ||
        (mode == 1 && (!x || !grad || !saved || !rws || !rblk || !rper || !gain || !lscore ||
                       !lflags || !ltws)))
        return fail(MPS_E_OUT_OF_MEMORY, "mps_search buffers");
    mps_moves ex{1, 1, 0, nullptr, nullptr};
    mps_moves lst{0, 1, k, rblk, rper};
    int64_t iters = 0, evals = 0, applied_total = 0;
    int32_t h_applied = 0;
    auto round_exhaustive = [&]() -> hipError_t {
        hipError_t e = launch_eval(d, ex, score, flags, nullptr, nullptr, nullptr, hs);
        if (e == hipSuccess)
            e = launch_topk(score, flags, nm, k, MPS_PREC_OK, MPS_NOOP | MPS_BAD, idx, nullptr,
                            cnt, tws, hs);
        if (e == hipSuccess)
            e = launch_repair(d, ex, idx, cnt, k, 0, cnt + 1, m->gather, m->rep_first, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&h_applied, cnt + 1, sizeof(int32_t), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        evals += nm;
        return e;
    };
    auto round_gradient = [&]() -> hipError_t {
        hipError_t e = launch_integer_x(d, x, hs);
        if (e == hipSuccess) e = launch_relaxed_fwd(d, x, *rp, nullptr, saved, m->relax_ws, hs);
        if (e == hipSuccess) e = launch_relaxed_bwd(d, x, *rp, saved, nullptr, grad, m->relax_ws, hs);
        if (e == hipSuccess) e = launch_rank(d, grad, k, rblk, rper, gain, cnt + 2, rws, hs);
        if (e == hipSuccess) e = launch_eval(d, lst, lscore, lflags, nullptr, nullptr, nullptr, hs);
        if (e == hipSuccess)
            e = launch_topk(lscore, lflags, k, k, MPS_PREC_OK, MPS_NOOP | MPS_BAD, idx, nullptr,
                            cnt, ltws, hs);
        if (e == hipSuccess)
            e = launch_repair(d, lst, idx, cnt, k, 0, cnt + 1, m->gather, m->rep_first, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&h_applied, cnt + 1, sizeof(int32_t), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        evals += k;
        return e;
    };
    hipError_t e = hipSuccess;
    while (iters < max_iter) {
        e = mode == 0 ? round_exhaustive() : round_gradient();
        if (e != hipSuccess) break;
        ++iters;
        applied_total += h_applied;
        if (h_applied == 0) {
            if (mode == 0) break;
            e = round_exhaustive();
            if (e != hipSuccess) break;
            ++iters;
            applied_total += h_applied;
            if (h_applied == 0) break;
        }
    }
    if (e != hipSuccess) return dev_fail(e, "search");
    mps_objective obj;
    if ((st = mps_get_objective(m, &obj, stream)) != MPS_OK) return st;
    if (out) {
        out->iterations = iters;
        out->evaluations = evals;
        out->applied = applied_total;
        out->J = obj.J;
    }
    return MPS_OK;
}

}  // extern "C"

// ---- batches -------------------------------------------------------------------
namespace {

std::mutex g_tune_mu;
std::map<int, mps_tuning> g_tune_cache;   // S class -> tuning chosen by the autotuner

int tune_class(int32_t S) { return S <= 32 ? 0 : S <= 64 ? 1 : S <= 128 ? 2 : 3; }

mps_tuning default_tuning(int32_t S) {
    mps_tuning t{};
    t.tiles_per_item = 2;
    t.moves_per_item = 4096;
    t.rows = S <= 64 ? 8 : S <= 128 ? 16 : 32;
    return t;
}

bool tuning_ok(const mps_tuning &t) {
    return t.reserved == 0 && t.tiles_per_item >= 1 && t.tiles_per_item <= 64 &&
           t.moves_per_item >= 512 && t.moves_per_item <= 65536 && t.moves_per_item % 512 == 0 &&
           (t.rows == 8 || t.rows == 16 || t.rows == 32);
}

}  // namespace

struct mps_batch {
    int device = 0;
    int32_t n = 0, k = 0;
    uint8_t req = 0, forbid = 0;
    std::vector<mps_model *> models;
    std::vector<mps_batch_item> items;
    std::vector<mps_tuning> tune;
    std::vector<int32_t> order;   // models by decreasing block-value bytes
    std::vector<int32_t *> perm;  // per model: block order of its moves (batch_sort_moves)
    std::vector<int32_t> perm_mpi;   // the range length each perm was sorted with
    BatchInst *d_insts = nullptr;
    int2 *d_items1 = nullptr, *d_items2 = nullptr;
    int32_t *d_order = nullptr;
    uint32_t *d_ctl = nullptr;
    int64_t max_items1 = 0, max_items2 = 0;
    int32_t n_items1 = 0, n_items2 = 0;
    size_t lds = 0;
    int per_cu = 1, cus = 1, workgroups = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    void drop_graph() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    int grid(int32_t items) const {
        const int full = per_cu * cus;
        int g = workgroups > 0 ? std::min(workgroups, full) : full;
        if ((int64_t)g > items) g = (int)items;
        return g > 0 ? g : 1;
    }
    BatchLaunch launch() const {
        BatchLaunch bl;
        bl.insts = d_insts;
        bl.items1 = d_items1;
        bl.items2 = d_items2;
        bl.order = d_order;
        bl.n_items1 = n_items1;
        bl.n_items2 = n_items2;
        bl.n_inst = n;
        bl.ctl = d_ctl;
        bl.k = k;
        bl.req = req;
        bl.forbid = forbid;
        bl.grid1 = grid(n_items1);
        bl.grid2 = grid(n_items2);
        // the top-k passes claim about 16K moves at a time
        int32_t mpi_min = 1 << 30;
        for (const mps_tuning &tu : tune) mpi_min = std::min(mpi_min, tu.moves_per_item);
        bl.claim = std::max(1, 16384 / std::max(1, mpi_min));
        bl.lds_bytes = lds;
        return bl;
    }
    // Descriptors and work queue from the current tuning (synchronous copies).
    mps_status rebuild() {
        std::vector<BatchInst> hi(n);
        for (int32_t i = 0; i < n; ++i) {
            const mps_batch_item &it = items[i];
            BatchInst &I = hi[i];
            I.m = models[i]->d;
            I.blk = it.block;
            I.per = it.period;
            I.perm = perm[i];
            I.n = it.n;
            I.score = it.score;
            I.flags = it.flags;
            I.top_idx = it.top_idx;
            I.top_score = it.top_score;
            I.top_count = it.top_count;
            I.n_tiles = (int32_t)((I.m.N + 63) / 64);
            I.tiles_per_item = tune[i].tiles_per_item;
            I.n1 = it.n > 0 ? (I.n_tiles + I.tiles_per_item - 1) / I.tiles_per_item : 0;
            I.moves_per_item = tune[i].moves_per_item;
            I.n2 = (int32_t)((it.n + I.moves_per_item - 1) / I.moves_per_item);
            I.rows = tune[i].rows;
        }
        {
            DeviceGuard g(device);
            for (int32_t i = 0; i < n; ++i) {
                // one sorted range per move item (longer ranges, which give
                // each item a contiguous stretch of blocks, measured slower:
                // the items of a range then write the same lines of scores
                // from different XCDs)
                const int32_t seg = hi[i].moves_per_item;
                if (items[i].n <= 0 || perm_mpi[i] == seg) continue;
                const hipError_t e =
                    batch_sort_moves(items[i].block, items[i].n, seg, perm[i], nullptr);
                if (e != hipSuccess) return dev_fail(e, "block order of a batch's moves");
                perm_mpi[i] = seg;
            }
        }
        std::vector<int2> q1, q2;
        for (int32_t i : order)
            for (int32_t j = 0; j < hi[i].n1; ++j) q1.push_back(make_int2(i, j));
        for (int32_t i : order)
            for (int32_t j = 0; j < hi[i].n2; ++j) q2.push_back(make_int2(i, j));
        if ((int64_t)q1.size() > max_items1 || (int64_t)q2.size() > max_items2)
            return fail(MPS_E_INTERNAL, "work queue overflow");
        DeviceGuard g(device);
        hipError_t e = hipMemcpy(d_insts, hi.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice);
        if (e == hipSuccess && !q1.empty())
            e = hipMemcpy(d_items1, q1.data(), sizeof(int2) * q1.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !q2.empty())
            e = hipMemcpy(d_items2, q2.data(), sizeof(int2) * q2.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d_order, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return dev_fail(e, "batch descriptors");
        n_items1 = (int32_t)q1.size();
        n_items2 = (int32_t)q2.size();
        drop_graph();
        return MPS_OK;
    }
    ~mps_batch() {
        DeviceGuard g(device);
        drop_graph();
        if (cap) hipStreamDestroy(cap);
        hipFree(d_insts);
        hipFree(d_items1);
        hipFree(d_items2);
        hipFree(d_order);
        hipFree(d_ctl);
        for (int32_t *p : perm) hipFree(p);
    }
};

extern "C" {

mps_status mps_batch_create(mps_model *const *models, const mps_batch_item *items,
                            int32_t n_models, int32_t k, uint8_t require, uint8_t forbid,
                            mps_batch **out) {
    if (!out) return fail(MPS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!models || !items) return fail(MPS_E_INVALID_ARG, "models and items are required");
    if (n_models < 1 || n_models > MPS_MAX_BATCH)
        return fail(MPS_E_INVALID_ARG, "n_models must be in 1..%d", MPS_MAX_BATCH);
    if (k < 1 || k > MPS_MAX_BATCH_TOPK)
        return fail(MPS_E_INVALID_ARG, "k must be in 1..%d (got %d)", MPS_MAX_BATCH_TOPK, k);
    size_t lds = 0;
    int64_t max_items1 = 0, max_items2 = 0;
    for (int32_t i = 0; i < n_models; ++i) {
        const mps_model *m = models[i];
        const mps_batch_item &it = items[i];
        if (!m) return fail(MPS_E_INVALID_ARG, "model %d is NULL", i);
        {
            const mps_status vs = no_variant(m, "mps_batch_create");
            if (vs != MPS_OK) return vs;
        }
        if (m->device != models[0]->device)
            return fail(MPS_E_INVALID_ARG, "model %d is on another device", i);
        if (it.n < 0 || it.n >= ((int64_t)1 << 31))
            return fail(MPS_E_INVALID_ARG, "item %d: n = %lld out of range", i, (long long)it.n);
        if (it.n > 0 && (!it.block || !it.period || !it.score || !it.flags))
            return fail(MPS_E_INVALID_ARG, "item %d: block, period, score, flags are required", i);
        if (!it.top_idx || !it.top_count)
            return fail(MPS_E_INVALID_ARG, "item %d: top_idx and top_count are required", i);
        lds = std::max(lds, batch_lds_bytes(m->d));
        max_items1 += (m->d.N + 63) / 64;
        max_items2 += (it.n + 511) / 512;
    }
    if (lds > (size_t)models[0]->max_lds)
        return fail(MPS_E_INVALID_ARG, "batch needs %zu bytes of LDS, device allows %d", lds,
                    models[0]->max_lds);
    if (max_items1 >= ((int64_t)1 << 31) || max_items2 >= ((int64_t)1 << 31))
        return fail(MPS_E_INVALID_ARG, "batch too large");
    mps_batch *b = new mps_batch;
    b->device = models[0]->device;
    b->n = n_models;
    b->k = k;
    b->req = require;
    b->forbid = forbid;
    b->models.assign(models, models + n_models);
    b->items.assign(items, items + n_models);
    b->lds = lds;
    b->max_items1 = max_items1;
    b->max_items2 = max_items2;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int32_t i = 0; i < n_models; ++i) {
            auto f = g_tune_cache.find(tune_class(models[i]->d.S));
            b->tune.push_back(f != g_tune_cache.end() ? f->second : default_tuning(models[i]->d.S));
        }
    }
    b->order.resize(n_models);
    for (int32_t i = 0; i < n_models; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t a, int32_t c) {
        const DevModel &x = models[a]->d, &y = models[c]->d;
        return (int64_t)x.S * x.N > (int64_t)y.S * y.N;
    });
    DeviceGuard g(b->device);
    hipError_t e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess) e = batch_occupancy(lds, &b->per_cu);
    if (e == hipSuccess && b->per_cu < 1) e = hipErrorInvalidConfiguration;
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_insts, sizeof(BatchInst) * n_models);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->d_items1, sizeof(int2) * (size_t)std::max<int64_t>(max_items1, 1));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->d_items2, sizeof(int2) * (size_t)std::max<int64_t>(max_items2, 1));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_order, sizeof(int32_t) * n_models);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->d_ctl, sizeof(uint32_t) * (size_t)batch_ctl_words(n_models));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    b->perm.assign(n_models, nullptr);
    b->perm_mpi.assign(n_models, 0);
    for (int32_t i = 0; i < n_models && e == hipSuccess; ++i)
        if (items[i].n > 0)
            e = hipMalloc((void **)&b->perm[i], sizeof(int32_t) * (size_t)items[i].n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return dev_fail(e, "batch create");
    }
    mps_status st = b->rebuild();
    if (st != MPS_OK) {
        delete b;
        return st;
    }
    *out = b;
    return MPS_OK;
}

mps_status mps_batch_destroy(mps_batch *b) {
    if (!b) return fail(MPS_E_INVALID_ARG, "batch is NULL");
    {
        DeviceGuard g(b->device);
        hipDeviceSynchronize();
    }
    delete b;
    return MPS_OK;
}

mps_status mps_batch_set_tuning(mps_batch *b, int32_t i, const mps_tuning *t) {
    if (!b || !t) return fail(MPS_E_INVALID_ARG, "batch and tuning are required");
    if (i < -1 || i >= b->n) return fail(MPS_E_INVALID_ARG, "model index %d out of range", i);
    if (!tuning_ok(*t))
        return fail(MPS_E_INVALID_ARG,
                    "tuning out of range (tiles_per_item 1..64, moves_per_item a multiple of "
                    "512 in 512..65536, rows 8/16/32, reserved 0)");
    if (i < 0) {
        std::fill(b->tune.begin(), b->tune.end(), *t);
        std::fill(b->perm_mpi.begin(), b->perm_mpi.end(), 0);   // order recomputed
    } else {
        b->tune[i] = *t;
        b->perm_mpi[i] = 0;
    }
    return b->rebuild();
}

mps_status mps_batch_get_tuning(const mps_batch *b, int32_t i, mps_tuning *t) {
    if (!b || !t) return fail(MPS_E_INVALID_ARG, "batch and tuning are required");
    if (i < 0 || i >= b->n) return fail(MPS_E_INVALID_ARG, "model index %d out of range", i);
    *t = b->tune[i];
    return MPS_OK;
}

mps_status mps_batch_set_workgroups(mps_batch *b, int32_t n) {
    if (!b) return fail(MPS_E_INVALID_ARG, "batch is NULL");
    if (n < 0 || n > b->per_cu * b->cus)
        return fail(MPS_E_INVALID_ARG, "workgroups must be in 0..%d", b->per_cu * b->cus);
    b->workgroups = n;
    b->drop_graph();
    return MPS_OK;
}

mps_status mps_batch_run(mps_batch *b, void *stream) {
    if (!b) return fail(MPS_E_INVALID_ARG, "batch is NULL");
    DeviceGuard g(b->device);
    hipError_t e = launch_batch(b->launch(), (hipStream_t)stream);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "batch run");
}

mps_status mps_batch_graph_launch(mps_batch *b, void *stream) {
    if (!b) return fail(MPS_E_INVALID_ARG, "batch is NULL");
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_batch_graph_launch during capture");
    DeviceGuard g(b->device);
    if (!b->exec) {
        hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return dev_fail(e, "begin capture");
        const hipError_t el = launch_batch(b->launch(), b->cap);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(b->cap, &gr);
        if (el != hipSuccess || e != hipSuccess) {
            if (gr) hipGraphDestroy(gr);
            return dev_fail(el != hipSuccess ? el : e, "capture batch");
        }
        b->graph = gr;
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->drop_graph();
            return dev_fail(e, "instantiate batch graph");
        }
    }
    hipError_t e = hipGraphLaunch(b->exec, hs);
    return e == hipSuccess ? MPS_OK : dev_fail(e, "launch batch graph");
}

mps_status mps_batch_autotune(mps_batch *b, int32_t reps, double *best_us, void *stream) {
    if (!b) return fail(MPS_E_INVALID_ARG, "batch is NULL");
    if (reps < 1 || reps > 1000) return fail(MPS_E_INVALID_ARG, "reps must be in 1..1000");
    hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(MPS_E_NOT_CAPTURABLE, "mps_batch_autotune during capture");
    DeviceGuard g(b->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return dev_fail(hipGetLastError(), "autotune events");
    }
    std::vector<float> ts(reps);
    // median time of `reps` runs (after one untimed run), in microseconds
    auto measure = [&](double &us) -> mps_status {
        hipError_t e = launch_batch(b->launch(), hs);
        for (int32_t r = 0; r < reps && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, hs);
            if (e == hipSuccess) e = launch_batch(b->launch(), hs);
            if (e == hipSuccess) e = hipEventRecord(e1, hs);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ts[r], e0, e1);
        }
        if (e != hipSuccess) return dev_fail(e, "autotune run");
        std::vector<float> t2 = ts;
        std::nth_element(t2.begin(), t2.begin() + reps / 2, t2.end());
        us = 1e3 * t2[reps / 2];
        return MPS_OK;
    };
    mps_status st = MPS_OK;
    double best = 0.0;
    std::vector<int> classes;
    for (int32_t i = 0; i < b->n; ++i) classes.push_back(tune_class(b->models[i]->d.S));
    std::sort(classes.begin(), classes.end());
    classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
    if ((st = measure(best)) != MPS_OK) goto done;
    for (int c : classes) {
        // one parameter at a time, the others held at their current best
        for (int param = 0; param < 3; ++param) {
            static const int kRows[] = {8, 16, 32};
            static const int kTiles[] = {1, 2, 4, 8};
            static const int kMoves[] = {1024, 2048, 4096, 8192, 16384, 32768};
            const int *vals = param == 0 ? kRows : param == 1 ? kTiles : kMoves;
            const int nv = param == 0 ? 3 : param == 1 ? 4 : 6;
            for (int v = 0; v < nv; ++v) {
                std::vector<mps_tuning> saved = b->tune;
                bool changed = false;
                for (int32_t i = 0; i < b->n; ++i) {
                    if (tune_class(b->models[i]->d.S) != c) continue;
                    mps_tuning &t = b->tune[i];
                    int &field = param == 0 ? t.rows : param == 1 ? t.tiles_per_item
                                                                  : t.moves_per_item;
                    if (field != vals[v]) changed = true;
                    field = vals[v];
                }
                if (!changed) continue;
                double us = 0.0;
                if ((st = b->rebuild()) != MPS_OK || (st = measure(us)) != MPS_OK) goto done;
                if (us < best) {
                    best = us;
                } else {
                    b->tune = saved;
                    if ((st = b->rebuild()) != MPS_OK) goto done;
                }
            }
        }
    }
    {
        const int full = b->per_cu * b->cus;
        const int cands[] = {b->cus, 2 * b->cus, 0};
        int best_wg = b->workgroups;
        for (int wg : cands) {
            if (wg > full || wg == b->workgroups) continue;
            const int old = b->workgroups;
            b->workgroups = wg;
            b->drop_graph();
            double us = 0.0;
            if ((st = measure(us)) != MPS_OK) goto done;
            if (us < best) {
                best = us;
                best_wg = wg;
            }
            b->workgroups = old;
        }
        b->workgroups = best_wg;
        b->drop_graph();
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int32_t i = 0; i < b->n; ++i) g_tune_cache[tune_class(b->models[i]->d.S)] = b->tune[i];
    }
    // leave the outputs those of the chosen tuning
    {
        double us = 0.0;
        st = measure(us);
    }
done:
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st == MPS_OK && best_us) *best_us = best;
    return st;
}

}  // extern "C"
