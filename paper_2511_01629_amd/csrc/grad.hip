// grad.hip -- differentiated runs: forward with checkpoints, then the
// hand-written adjoint swept backwards segment by segment.
//
// Every adjoint step n needs the populations that entered step n and the
// indicator of step n ("frame" n), plus the step's particle record.
//
// every > 1: the forward run snapshots the whole state (populations,
// indicator, particle arrays) every `every` steps.  The backward pass restores
// a segment's snapshot into the first of every + 1 frames and recomputes the
// segment with step n reading frame n and writing frame n + 1 directly, both
// the populations and the indicator (the indicator frames are filled with
// FLUID first, so the step rasterises into a clean map and no copy is made);
// then it runs the segment's adjoint steps in reverse.  All kernels are
// deterministic, so the recomputed frames are bitwise those of the forward run.
//
// every == 1: the forward run itself writes every frame (T + 1 population
// buffers and T + 1 indicators -- e.g. 100 GB for 5000 steps of a 512x1024
// FP32 lattice, which 288 GB of HBM holds), and the backward pass recomputes
// nothing.
#include <algorithm>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "ctx.h"

using namespace lbm;

struct GradState {
    // the particle set and slot layout the run was recorded with
    int np = 0, fused = 0, slot_stride = 0;
    int64_t T = 0;
    int every = 0, nsnap = 0;
    size_t fbytes = 0, obytes = 0, pbytes = 0;
    char *snap = nullptr;  // nsnap x (fbytes + obytes + pbytes)
    char *hist = nullptr;  // every == 1: (T + 1) population frames, then T + 1 indicators
    std::vector<PartDev> snapP;
    std::vector<int> snapCur;
    std::vector<int64_t> snapStep;
    double *rec = nullptr; // T x np x REC_STRIDE
    std::vector<double> gX0; // dL/dX^0 of the last backward sweep, [np][3] (empty before one)
    std::vector<void *> owned; // library allocations (none when the caller supplied the memory)
};

namespace {

// A roctx range over a scope: the phases of a differentiated run (forward,
// each segment's recomputation and adjoint sweep) as host-side ranges in a
// rocprofv3 --marker-trace timeline.  The ranges mark when the host queues
// the work; the kernels they enclose run on the device afterwards.
struct Range {
    explicit Range(const char *m) { roctxRangePush(m); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

#define HIPCHK(c, expr)                                                                                                \
    do {                                                                                                               \
        hipError_t e_ = (expr);                                                                                        \
        if (e_ != hipSuccess) {                                                                                        \
            (c)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                                              \
            return LBM_EDEVICE;                                                                                        \
        }                                                                                                              \
    } while (0)

size_t storage_bytes(int s) { return s == LBM_F64 ? 8 : s == LBM_F32 ? 4 : 2; }

// The particle arrays occupy one contiguous region of the workspace, from
// P.X's block start (the first double array) to the end of the int block.
char *part_base(lbm_ctx *c) { return (char *)std::min(c->P.X, c->P.Xn); }
size_t part_bytes(lbm_ctx *c) { return (size_t)((char *)(c->P.hi + 3 * c->cap) - part_base(c)); }

int snapshot(lbm_ctx *c, GradState *G, int k)
{
    char *dst = G->snap + (size_t)k * (G->fbytes + G->obytes + G->pbytes);
    HIPCHK(c, hipMemcpyAsync(dst, c->f[c->cur], G->fbytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dst + G->fbytes, c->owner, G->obytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dst + G->fbytes + G->obytes, part_base(c), G->pbytes, hipMemcpyDeviceToDevice, c->stream));
    G->snapP[k] = c->P;
    G->snapCur[k] = c->cur;
    G->snapStep[k] = c->step;
    return LBM_OK;
}

// Restore snapshot k; its populations go to fdst and its indicator to odst
// (NULL: the live buffers).
int restore(lbm_ctx *c, GradState *G, int k, void *fdst = nullptr, void *odst = nullptr)
{
    const char *src = G->snap + (size_t)k * (G->fbytes + G->obytes + G->pbytes);
    c->P = G->snapP[k];
    c->cur = G->snapCur[k];
    c->step = G->snapStep[k];
    HIPCHK(c, hipMemcpyAsync(fdst ? fdst : c->f[c->cur], src, G->fbytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(odst ? odst : c->owner, src + G->fbytes, G->obytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(part_base(c), src + G->fbytes + G->obytes, G->pbytes, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

// Steps s0 .. s0 + n - 1 with step s reading population frame s - s0 of fr and
// indicator frame s - s0 of ow, and writing frame s - s0 + 1 of each.
// Indicator frames 1 .. n are filled with FLUID first; frame 0 must hold the
// indicator of step s0.  rec (optional): the particle records of the steps.
// The live buffers are restored afterwards (the caller copies what it keeps).
int run_frames(lbm_ctx *c, GradState *G, char *fr, char *ow, int64_t n, double *rec)
{
    HIPCHK(c, hipMemsetAsync(ow + G->obytes, 0xFF, (size_t)n * G->obytes, c->stream));
    uint16_t *live = c->owner;
    int rc = LBM_OK;
    for (int64_t s = 0; s < n && rc == LBM_OK; ++s) {
        c->f[c->cur] = fr + (size_t)s * G->fbytes;
        c->f[c->cur ^ 1] = fr + (size_t)(s + 1) * G->fbytes;
        c->owner = (uint16_t *)(ow + (size_t)s * G->obytes);
        c->owner_next = (uint16_t *)(ow + (size_t)(s + 1) * G->obytes);
        rc = step_impl(c, 1, rec ? rec + (size_t)s * c->np * REC_STRIDE : nullptr);
    }
    c->f[0] = c->fws[0];
    c->f[1] = c->fws[1];
    c->owner = live;
    c->owner_next = nullptr;
    return rc;
}

// The memory of a differentiated run, taken piece by piece (each 256-byte
// aligned): allocated by the library (base == NULL, count == false; freed with
// the run), carved from a caller's buffer of `cap` bytes (never freed here),
// or only counted (count == true: a size query).
struct Carver {
    lbm_ctx *c;
    char *base;
    size_t cap;
    bool count;
    std::vector<void *> *owned;
    size_t off = 0;

    template <class Tp> int take(Tp **p, size_t n, bool zero)
    {
        const size_t bytes = (std::max<size_t>(n, 1) * sizeof(Tp) + 255) / 256 * 256;
        *p = nullptr;
        if (count) {
            off += bytes;
            return LBM_OK;
        }
        if (base) {
            if (off + bytes > cap) return c->err = "the caller's workspace is too small", LBM_ENOMEM;
            *p = (Tp *)(base + off);
        } else {
            const hipError_t e = hipMalloc((void **)p, bytes);
            if (e != hipSuccess) return c->err = std::string("hipMalloc: ") + hipGetErrorString(e), LBM_ENOMEM;
            owned->push_back(*p);
        }
        off += bytes;
        if (zero) HIPCHK(c, hipMemsetAsync(*p, 0, bytes, c->stream));
        return LBM_OK;
    }
};

// Frame strides, rounded up to the 256 bytes the context's own buffers are
// aligned to (and sized to): frames sit back to back in the segment and
// history buffers, and the rasterisation claims indicator entries with 32-bit
// compare-and-swap, so every indicator frame must start on a 4-byte boundary
// -- which Q N s bytes of 2-byte populations with Q N odd would break.
size_t round_frame(size_t v) { return (v + 255) / 256 * 256; }
// The lattice adjoint keeps 32-bit population offsets.
bool narrow_offsets(const lbm_ctx *c) { return (int64_t)c->Q * c->geo.N < ((int64_t)1 << 31); }
const char *const WIDE_MSG = "the differentiated run keeps 32-bit population offsets: Q*N must stay below 2^31";

size_t frame_bytes(const lbm_ctx *c) { return round_frame((size_t)c->Q * c->geo.N * storage_bytes(c->cfg.storage)); }
size_t owner_bytes(const lbm_ctx *c) { return round_frame((size_t)((c->geo.N + 1) / 2 * 2) * sizeof(uint16_t)); }

// The forward run's pieces: the particle records, then the frames (every = 1)
// or the snapshots.
int carve_forward(Carver &m, int64_t T, int every, size_t fbytes, size_t obytes, size_t pbytes, double **rec,
                  char **hist, char **snap)
{
    const int nsnap = (int)((T + every - 1) / every) + 1;
    *hist = *snap = nullptr;
    int rc = m.take(rec, (size_t)T * m.c->np * REC_STRIDE, false);
    if (!rc && every == 1) rc = m.take(hist, (size_t)(T + 1) * (fbytes + obytes), false);
    if (!rc && every > 1) rc = m.take(snap, (size_t)nsnap * (fbytes + obytes + pbytes), false);
    return rc;
}

// The backward sweep's pieces (lbm_backward): per-(particle, slot) records of
// the a_bar sums where the forward step has slots; one or two segment buffers
// of every + 1 frames; particle constants; the two adjoint population
// buffers; the per-node a_bar field (without slots); per-workgroup tau
// partials; the particle adjoints.
struct BackBufs {
    double *aslots = nullptr;
    char *seg = nullptr, *seg2 = nullptr, *lam = nullptr;
    double *cst = nullptr;
    int32_t *cshape = nullptr;
    double *asol = nullptr, *taup = nullptr, *Xbar = nullptr, *Abar = nullptr, *Upbar = nullptr, *rho_g = nullptr,
           *g_g = nullptr, *uext_d = nullptr, *acc_d = nullptr;
    float *uext_f = nullptr, *acc_f = nullptr;
    double *fpart = nullptr, *geo = nullptr; // fractional indicator only
};

int carve_backward(Carver &m, int64_t T, int every, size_t fbytes, size_t obytes, BackBufs &b)
{
    lbm_ctx *c = m.c;
    const int np = c->np, Q = c->Q;
    const int64_t N = c->geo.N;
    const size_t lam_elt = c->cfg.storage == LBM_F64 ? 8 : 4;
    const size_t nblocks = (size_t)((c->geo.nx + 255) / 256) * c->geo.ny * c->geo.nz;
    const bool all = every == 1;
    const int nseg = all ? 1 : (int)((T + every - 1) / every);
    const bool overlap = !all && nseg > 1;
    const size_t segsize = all ? 1 : (size_t)(every + 1) * (fbytes + obytes); // every + 1 frames of each
    const bool slots = c->fused && c->slots && np > 0;
    int rc = LBM_OK;
    if (slots) rc = m.take(&b.aslots, (size_t)np * (size_t)c->slot_stride * (size_t)(c->d + 1), false);
    if (!rc) rc = m.take(&b.seg, segsize, true);
    if (!rc && overlap) rc = m.take(&b.seg2, segsize, true);
    if (!rc) rc = m.take(&b.cst, 4 * (size_t)np, true);
    if (!rc) rc = m.take(&b.cshape, (size_t)np, true);
    if (!rc) rc = m.take(&b.lam, 2 * Q * N * lam_elt, true);
    // a_bar per node, and with the fractional indicator chi_bar dchi/dX
    if (!rc) rc = m.take(&b.asol, slots ? 1 : (size_t)c->d * N * (c->sp.frac ? 2 : 1), true);
    if (!rc) rc = m.take(&b.taup, nblocks, true);
    if (!rc) rc = m.take(&b.Xbar, 6 * (size_t)np, true);
    if (!rc) rc = m.take(&b.Abar, 3 * (size_t)np, true);
    if (!rc) rc = m.take(&b.Upbar, 6 * (size_t)np, true);
    if (!rc) rc = m.take(&b.rho_g, np, true);
    if (!rc) rc = m.take(&b.g_g, np, true);
    if (!rc) rc = m.take(&b.uext_d, 3 * (size_t)np, true);
    if (!rc) rc = m.take(&b.acc_d, 3 * (size_t)np, true);
    if (!rc) rc = m.take(&b.uext_f, 3 * (size_t)np, true);
    if (!rc) rc = m.take(&b.acc_f, 3 * (size_t)np, true);
    if (!rc && c->sp.frac) rc = m.take(&b.fpart, FRAC_STRIDE * (size_t)np, true);
    if (!rc && c->sp.frac) rc = m.take(&b.geo, 4 * (size_t)np, true);
    return rc;
}

int forward_impl(lbm_ctx *c, int64_t nsteps, int32_t every, void *ws, size_t ws_bytes);
int backward_impl(lbm_ctx *c, const double *dL_dX, double *g_rho_s, double *g_tau, double *g_gmag, void *ws,
                  size_t ws_bytes);

} // namespace

void lbm::free_grad(lbm_ctx *c)
{
    if (!c->grad) return;
    (void)hipStreamSynchronize(c->stream);
    for (void *p : c->grad->owned) (void)hipFree(p);
    delete c->grad;
    c->grad = nullptr;
}

extern "C" {

int lbm_forward_checkpointed(lbm_ctx *c, int64_t nsteps, int32_t every)
{
    return c ? forward_impl(c, nsteps, every, nullptr, 0) : LBM_EINVAL;
}

int lbm_forward_checkpointed_ws(lbm_ctx *c, int64_t nsteps, int32_t every, void *ws, size_t ws_bytes)
{
    if (!c) return LBM_EINVAL;
    if (!ws) return c->err = "workspace is NULL", LBM_EINVAL;
    if ((uintptr_t)ws % 256) return c->err = "workspace is not 256-byte aligned", LBM_EINVAL;
    return forward_impl(c, nsteps, every, ws, ws_bytes);
}

int lbm_backward_ws(lbm_ctx *c, const double *dL_dX, double *g_rho_s, double *g_tau, double *g_gmag, void *ws,
                    size_t ws_bytes)
{
    if (!c || !dL_dX) return LBM_EINVAL;
    if (!ws) return c->err = "workspace is NULL", LBM_EINVAL;
    if ((uintptr_t)ws % 256) return c->err = "workspace is not 256-byte aligned", LBM_EINVAL;
    return backward_impl(c, dL_dX, g_rho_s, g_tau, g_gmag, ws, ws_bytes);
}

int lbm_grad_workspace_size(lbm_ctx *c, int64_t nsteps, int32_t every, size_t *fwd_bytes, size_t *bwd_bytes)
{
    if (!c) return LBM_EINVAL;
    if (nsteps < 1 || every < 1) return c->err = "nsteps and every must be >= 1", LBM_EINVAL;
    if (!narrow_offsets(c)) return c->err = WIDE_MSG, LBM_EINVAL;
    const size_t fb = frame_bytes(c), ob = owner_bytes(c);
    Carver f{c, nullptr, 0, true, nullptr};
    double *rec;
    char *hist, *snap;
    carve_forward(f, nsteps, every, fb, ob, part_bytes(c), &rec, &hist, &snap);
    Carver b{c, nullptr, 0, true, nullptr};
    BackBufs bb;
    carve_backward(b, nsteps, every, fb, ob, bb);
    if (fwd_bytes) *fwd_bytes = f.off;
    if (bwd_bytes) *bwd_bytes = b.off;
    return LBM_OK;
}

} // extern "C"

namespace {

int forward_impl(lbm_ctx *c, int64_t nsteps, int32_t every, void *ws, size_t ws_bytes)
{
    Range range("lbm forward (checkpointed)");
    if (nsteps < 1 || every < 1) return c->err = "nsteps and every must be >= 1", LBM_EINVAL;
    if (!narrow_offsets(c)) return c->err = WIDE_MSG, LBM_EINVAL;
    if (!c->fresh) return c->err = "a differentiated run must start right after lbm_set_particles", LBM_ESTATE;
    if (c->np == 0) return c->err = "no particles", LBM_ESTATE;
    if (c->rp.K != 1) return c->err = "the adjoint of Algorithm 1 is implemented for K = 1", LBM_EINVAL;
    if (c->sp.beta > 0 || !c->sp.stress)
        return c->err = "the adjoint covers the paper's method (no rigid-velocity forcing, stress penalty on)",
               LBM_EINVAL;
    (void)hipSetDevice(c->device);
    free_grad(c);
    GradState *G = new GradState();
    c->grad = G;
    G->np = c->np;
    G->fused = c->fused;
    G->slot_stride = c->slot_stride;
    G->T = nsteps;
    G->every = every;
    G->nsnap = (int)((nsteps + every - 1) / every) + 1; // segment starts + final state
    G->fbytes = frame_bytes(c);
    G->obytes = owner_bytes(c);
    G->pbytes = part_bytes(c);
    {
        Carver m{c, (char *)ws, ws_bytes, false, &G->owned};
        const int rc = carve_forward(m, nsteps, every, G->fbytes, G->obytes, G->pbytes, &G->rec, &G->hist, &G->snap);
        if (rc) {
            free_grad(c);
            return rc;
        }
    }
    if (every == 1) {
        // keep every frame: step n reads frame n and writes frame n + 1
        char *fr = G->hist, *ow = G->hist + (size_t)(nsteps + 1) * G->fbytes;
        HIPCHK(c, hipMemcpyAsync(fr, c->f[c->cur], G->fbytes, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(ow, c->owner, G->obytes, hipMemcpyDeviceToDevice, c->stream));
        int rc = run_frames(c, G, fr, ow, nsteps, G->rec);
        if (rc) return rc;
        // the final state back into the live buffers
        HIPCHK(c, hipMemcpyAsync(c->f[c->cur], fr + (size_t)nsteps * G->fbytes, G->fbytes, hipMemcpyDeviceToDevice,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(c->owner, ow + (size_t)nsteps * G->obytes, G->obytes, hipMemcpyDeviceToDevice,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return lbm_sync(c);
    }
    G->snapP.resize(G->nsnap);
    G->snapCur.resize(G->nsnap);
    G->snapStep.resize(G->nsnap);
    for (int64_t s = 0; s < nsteps; ++s) {
        if (s % every == 0) {
            int rc = snapshot(c, G, (int)(s / every));
            if (rc) return rc;
        }
        int rc = step_impl(c, 1, G->rec + (size_t)s * c->np * REC_STRIDE);
        if (rc) return rc;
    }
    int rc = snapshot(c, G, G->nsnap - 1);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return lbm_sync(c);
}

int backward_impl(lbm_ctx *c, const double *dL_dX, double *g_rho_s, double *g_tau, double *g_gmag, void *ws,
                  size_t ws_bytes)
{
    Range range("lbm backward");
    GradState *G = c->grad;
    if (!G) return c->err = "no differentiated forward run to go back through", LBM_ESTATE;
    if (G->np != c->np || G->fused != c->fused || G->slot_stride != c->slot_stride)
        return c->err = "the particles changed since the differentiated forward run", LBM_ESTATE;
    (void)hipSetDevice(c->device);
    const int np = c->np, Q = c->Q;
    const int64_t N = c->geo.N;
    const size_t lam_elt = c->cfg.storage == LBM_F64 ? 8 : 4;
    const int gx = (c->geo.nx + 255) / 256;
    const size_t nblocks = (size_t)gx * c->geo.ny * c->geo.nz;
    std::vector<void *> owned;
    const hipStream_t main_stream = c->stream;
    // every > 1 with several segments: segment s - 1 is recomputed on a second
    // stream (default priority) into the other of two segment buffers while
    // the adjoint sweeps segment s; events order the two.
    hipStream_t side = nullptr;
    hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    bool freed_set[2] = {false, false};
    auto cleanup = [&]() {
        c->stream = main_stream;
        (void)hipStreamSynchronize(main_stream);
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        for (int b = 0; b < 2; ++b) {
            if (ready[b]) (void)hipEventDestroy(ready[b]);
            if (freed[b]) (void)hipEventDestroy(freed[b]);
        }
        for (void *p : owned) (void)hipFree(p);
    };
    const bool all = G->hist != nullptr;
    const int nseg = all ? 1 : G->nsnap - 1;
    const bool overlap = !all && nseg > 1;
    int rc = LBM_OK;
    BackBufs bb;
    {
        Carver m{c, (char *)ws, ws_bytes, false, &owned};
        if ((rc = carve_backward(m, G->T, G->every, G->fbytes, G->obytes, bb))) {
            cleanup();
            return rc;
        }
    }
    char *seg = bb.seg, *seg2 = bb.seg2, *lam = bb.lam;
    double *cst = bb.cst;
    int32_t *cshape = bb.cshape;
    double *asol = bb.asol, *taup = bb.taup, *Xbar = bb.Xbar, *Abar = bb.Abar, *Upbar = bb.Upbar, *rho_g = bb.rho_g,
           *g_g = bb.g_g, *uext_d = bb.uext_d, *acc_d = bb.acc_d;
    float *uext_f = bb.uext_f, *acc_f = bb.acc_f;
    // per-(particle, slot) records of the lattice adjoint's a_bar sums, where
    // the forward step has a slot layout (else a_bar goes to asol per node)
    double *aslots = bb.aslots;
    int64_t astamp = 0;
    if (aslots && hipMemsetAsync(aslots, 0xFF, (size_t)np * c->slot_stride * (c->d + 1) * sizeof(double),
                                 c->stream) != hipSuccess) { // NaN stamps: no record counts until a step writes it
        cleanup();
        return c->err = "slot initialisation failed", LBM_EDEVICE;
    }
    // the particle constants the adjoint kernels read, in memory of their own
    // (a snapshot restore on the side stream rewrites the workspace copies)
    PartDev Pc = c->P;
    Pc.rho_s = cst;
    Pc.a = cst + np;
    Pc.b = cst + 2 * np;
    Pc.Cc = cst + 3 * np;
    Pc.shape = cshape;
    if (hipMemcpyAsync(Pc.rho_s, c->P.rho_s, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(Pc.a, c->P.a, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(Pc.b, c->P.b, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(Pc.Cc, c->P.Cc, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(Pc.shape, c->P.shape, np * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
        cleanup();
        return c->err = "constant copy failed", LBM_EDEVICE;
    }
    if (overlap) {
        bool ok = hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess;
        for (int b = 0; b < 2 && ok; ++b)
            ok = hipEventCreateWithFlags(&ready[b], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&freed[b], hipEventDisableTiming) == hipSuccess;
        // the side stream starts after everything queued so far on the main one
        ok = ok && hipEventRecord(freed[1], main_stream) == hipSuccess &&
             hipStreamWaitEvent(side, freed[1], 0) == hipSuccess;
        if (!ok) {
            cleanup();
            return c->err = "stream or event creation failed", LBM_EDEVICE;
        }
    }
    char *segbuf[2] = {seg, overlap ? seg2 : seg};
    const int64_t span = all ? G->T : G->every;
    // recompute segment sg into its buffer on the side stream
    auto recompute = [&](int sg) -> int {
        Range rr("lbm backward: recompute segment");
        const int b = sg & 1;
        char *fr = segbuf[b], *ow = segbuf[b] + (size_t)(G->every + 1) * G->fbytes;
        const int64_t s0 = (int64_t)sg * span, s1 = std::min<int64_t>(s0 + span, G->T);
        if (freed_set[b] && hipStreamWaitEvent(side, freed[b], 0) != hipSuccess) return LBM_EDEVICE;
        c->stream = side;
        int r = restore(c, G, sg, fr, ow);
        if (r == LBM_OK) r = run_frames(c, G, fr, ow, s1 - s0, nullptr);
        c->stream = main_stream;
        if (r == LBM_OK && hipEventRecord(ready[b], side) != hipSuccess) r = LBM_EDEVICE;
        return r;
    };

    // seed: X_bar^T = dL/dX_final; everything else zero
    std::vector<double> seed(3 * (size_t)np, 0.0);
    for (int i = 0; i < np; ++i)
        for (int k = 0; k < c->d; ++k) seed[3 * i + k] = dL_dX[3 * i + k];
    if (hipMemcpyAsync(Xbar, seed.data(), seed.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        cleanup();
        return c->err = "seed copy failed", LBM_EDEVICE;
    }
    int cx = 0, cu = 0, cl = 0; // which half of the ping-pong adjoint buffers is current
    // arrays of the rigid adjoint of step n (X_bar and the adjoint of U ping-pong)
    auto rigid_arrays = [&](int64_t n) {
        return AdjArraysHost{G->rec + (size_t)n * np * REC_STRIDE,
                             Xbar + 3 * np * cx,
                             Abar,
                             Upbar + 3 * np * cu,
                             Xbar + 3 * np * (cx ^ 1),
                             Upbar + 3 * np * (cu ^ 1),
                             uext_d,
                             uext_f,
                             acc_d,
                             acc_f,
                             rho_g,
                             g_g,
                             bb.fpart,
                             bb.geo};
    };
    if (overlap) rc = recompute(nseg - 1);
    for (int sg = nseg - 1; sg >= 0 && rc == LBM_OK; --sg) {
        const int64_t s0 = (int64_t)sg * span, s1 = std::min<int64_t>(s0 + span, G->T);
        char *fr, *ow; // frame n - s0 of populations / indicators
        if (all) {
            fr = G->hist;
            ow = G->hist + (size_t)(G->T + 1) * G->fbytes;
        } else if (overlap) {
            // queue the next segment's recomputation first, then this segment's sweep
            if (sg >= 1 && (rc = recompute(sg - 1))) break;
            if (hipStreamWaitEvent(main_stream, ready[sg & 1], 0) != hipSuccess) {
                rc = LBM_EDEVICE;
                break;
            }
            fr = segbuf[sg & 1];
            ow = fr + (size_t)(G->every + 1) * G->fbytes;
        } else {
            fr = seg;
            ow = seg + (size_t)(G->every + 1) * G->fbytes;
            Range rr("lbm backward: recompute segment");
            if ((rc = restore(c, G, sg, fr, ow))) break;
            if ((rc = run_frames(c, G, fr, ow, s1 - s0, nullptr))) break;
        }
        Range rs("lbm backward: adjoint sweep of a segment");
        for (int64_t n = s1 - 1; n >= s0 && rc == LBM_OK; --n) {
            const char *fprev = fr + (size_t)(n - s0) * G->fbytes;
            const uint16_t *own_n = (const uint16_t *)(ow + (size_t)(n - s0) * G->obytes);
            const double *rec_n = G->rec + (size_t)n * np * REC_STRIDE;
            // with slots the rigid adjoint of step n ran with the particle adjoint of step n + 1
            if (!aslots || n == G->T - 1) {
                if (launch_adj_rigid(c, Pc, rigid_arrays(n)) != hipSuccess) rc = LBM_EDEVICE;
                cx ^= 1;
                cu ^= 1;
            }
            char *lin = lam + (size_t)cl * Q * N * lam_elt, *lout = lam + (size_t)(cl ^ 1) * Q * N * lam_elt;
            SlotParams asl{};
            if (aslots) {
                asl = slot_params(c, true);
                asl.slots = aslots;
                asl.stamp = (double)(++astamp);
                asl.clear = nullptr;
            }
            if (rc == LBM_OK && launch_adj_lattice(c, fprev, own_n, uext_d, uext_f, acc_d, acc_f, lin, lout,
                                                   aslots ? nullptr : asol, taup, asl, bb.fpart, bb.geo,
                                                   n == 0) != hipSuccess)
                rc = LBM_EDEVICE;
            cl ^= 1;
            if (aslots) {
                // A_bar^n from the records, then the rigid adjoint of step n - 1
                const int rigid = n > 0;
                if (rc == LBM_OK &&
                    launch_adj_fused(c, Pc, rigid_arrays(rigid ? n - 1 : 0), asl, Abar, rigid) != hipSuccess)
                    rc = LBM_EDEVICE;
                if (rigid) {
                    cx ^= 1;
                    cu ^= 1;
                }
            } else if (rc == LBM_OK && launch_adj_particles(c, Pc, own_n, asol, rec_n, Abar, rho_g, g_g,
                                                            Xbar + 3 * np * cx) != hipSuccess) {
                rc = LBM_EDEVICE; // X_bar^n (the rigid adjoint of step n wrote it) gains the indicator's terms
            }
        }
        if (overlap && rc == LBM_OK) {
            // this segment's buffer may be recomputed into once its sweep is done
            if (hipEventRecord(freed[sg & 1], main_stream) != hipSuccess) rc = LBM_EDEVICE;
            freed_set[sg & 1] = true;
        }
    }
    // the initial U^{-1} (binary indicator; with the fractional one its terms
    // were taken by the lattice adjoint of step 0)
    if (rc == LBM_OK && !c->sp.frac && launch_adj_initial(c, Pc, Upbar + 3 * np * cu, rho_g, g_g) != hipSuccess)
        rc = LBM_EDEVICE;
    std::vector<double> hr(np), hg(np), ht(nblocks), hx(3 * (size_t)np);
    G->gX0.clear();
    if (rc == LBM_OK) {
        if (hipMemcpyAsync(hr.data(), rho_g, np * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipMemcpyAsync(hx.data(), Xbar + 3 * np * cx, hx.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess ||
            hipMemcpyAsync(hg.data(), g_g, np * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipMemcpyAsync(ht.data(), taup, nblocks * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            rc = LBM_EDEVICE;
    }
    if (rc == LBM_OK) {
        double gt = 0.0, gg = 0.0;
        for (size_t b = 0; b < nblocks; ++b) gt += ht[b];
        for (int i = 0; i < np; ++i) gg += hg[i];
        if (g_rho_s)
            for (int i = 0; i < np; ++i) g_rho_s[i] = hr[i];
        if (g_tau) *g_tau = gt;
        if (g_gmag) *g_gmag = gg;
        G->gX0 = hx;
    }
    c->f[0] = c->fws[0];
    c->f[1] = c->fws[1];
    int rr = all ? LBM_OK : restore(c, G, G->nsnap - 1);
    cleanup();
    if (rc != LBM_OK) {
        if (c->err.empty()) c->err = "adjoint kernel launch failed";
        return rc;
    }
    return rr;
}

} // namespace

extern "C" int lbm_backward(lbm_ctx *c, const double *dL_dX, double *g_rho_s, double *g_tau, double *g_gmag)
{
    if (!c || !dL_dX) return LBM_EINVAL;
    return backward_impl(c, dL_dX, g_rho_s, g_tau, g_gmag, nullptr, 0);
}

extern "C" int lbm_grad_positions(lbm_ctx *c, double *g_X0)
{
    if (!c || !g_X0) return LBM_EINVAL;
    if (!c->grad || c->grad->gX0.empty() || c->grad->np != c->np)
        return c->err = "no backward sweep to read the position gradient of", LBM_ESTATE;
    for (size_t i = 0; i < c->grad->gX0.size(); ++i) g_X0[i] = c->grad->gX0[i];
    return LBM_OK;
}

