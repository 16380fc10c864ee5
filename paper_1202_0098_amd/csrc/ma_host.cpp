// Host side of libmarnoldi: the C interface declared in include/marnoldi.h.
//
// ma_build_system validates the block-sparse pencil, builds the real-space
// region of every atom (Sec. 3 of arXiv:1202.0098: H and S are projected on a
// sphere, or the N_RP nearest atoms, around the atom of basis j), the local
// block index of every region, and uploads FP64 and FP32 copies of H and S.
// ma_solve_columns orders the columns largest region first, launches the
// persistent column kernel, the chemical-potential bisection and the
// Fermi-weighting pass, and reduces the scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/marnoldi.h"
#include "ma_internal.h"

namespace {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow to at least n bytes (contents are not preserved)
    hipError_t reserve(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n ? n : 16);
        if (e == hipSuccess) bytes = n ? n : 16;
        return e;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

template <typename F>
void parallel_for(int64_t n, F &&f)
{
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    if (n < 64 || nt == 1) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    std::atomic<int64_t> next(0);
    const int64_t chunk = std::max<int64_t>(1, n / (nt * 16));
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (;;) {
                int64_t b = next.fetch_add(chunk);
                if (b >= n) break;
                f(b, std::min(n, b + chunk), (int)t);
            }
        });
    for (auto &x : th) x.join();
}

}  // namespace

struct ma_ctx {
    int device = 0;
    hipStream_t stream = nullptr;     // the caller's stream
    hipStream_t own = nullptr;        // used instead when the caller's is the null stream
    hipStream_t aux = nullptr;        // eigensolver of chunk k beside the basis kernel of chunk k+1
    hipStream_t aux2 = nullptr;       // eigensolver of the last chunk, beside the one before it
    hipEvent_t evu = nullptr;         // orders `own` after the caller's null stream
    // the stream the solve path enqueues on (the null stream cannot be captured)
    hipStream_t work_stream() const { return stream ? stream : own; }
    // Order the library's stream after the work already queued on the
    // caller's stream (needed whenever they differ: the caller's device
    // arrays may still be being written there).
    hipError_t after_caller()
    {
        if (stream) return hipSuccess;
        hipError_t e = hipEventRecord(evu, nullptr);
        if (e == hipSuccess) e = hipStreamWaitEvent(own, evu, 0);
        return e;
    }
    std::string err = "no error";
    int cu_count = 0;
    bool built = false;

    // system sizes
    int o = 0, n_atoms = 0;
    int64_t nblk = 0, M = 0;
    int nmax = 0, maxpat = 0, max_nat = 0;
    int64_t max_lnnz = 0;
    std::vector<int32_t> reg_len_of_atom;   // host: region atoms per atom (for ordering)
    std::vector<int32_t> spatial_rank;      // host: each atom's place in Morton order (MA_SCHED_SPATIAL)
    std::vector<int64_t> lblk_of_atom;      // host: local operator blocks per atom
    std::vector<int32_t> pat_blocks;        // host: blocks in each atom's block-row

    // device system
    DevBuf blk_t;                     // per block (A, B): the index of block (B, A)
    DevBuf reg_atoms;                 // the atoms of every region (ascending per region)
    // kept s_j (opts.keep_sj) and the regions of the geometry they belong to
    DevBuf sj_store, sj_have, sj_reg_id, sj_reg_off, sj_reg_len, sj_reg_atoms, x0full;
    bool sj_valid = false;
    uint64_t sj_gen = 0;
    int sj_nmax = 0, sj_n_atoms = 0, sj_o = 0;
    int64_t sj_nreg = 0, sj_natoms_total = 0;
    int64_t nreg = 0, reg_atoms_total = 0;
    DevBuf dos_E, dos_part, dos_out;  // density-of-states buffers
    DevBuf blk_ptr, blk_col, Hd, Sd, Hf, Sf, reg_id, reg_off, reg_len, lrp_off, lrp, lblk, jloc,
        blk_loc;
    bool have_geo = false;            // neighbour descriptors were built
    DevBuf geo, out_loc;              // n_atoms * kGeoFeat floats; n_atoms * kNbOut ints

    // start network: FP32 parameters, Adam moments, BF16 transposed weights,
    // training workspace
    struct Model {
        bool ready = false, bf16_dirty = true;
        int nf = 0, nh = 0, no = 0, nf_pad = 0, no_pad = 0, step = 0;
        int64_t P = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
        DevBuf params, grad, m, v, W1t, W2t, W3t;
        DevBuf Xb, Tb, Z1, A1, Z2, A2, Yb, dY, dA, partial, bad;
    } net;
    DevBuf feat, x0;                  // per-solve descriptors and predicted starts

    // device solve buffers
    DevBuf cols, order, qbounds, gstart, ws, eps, wts, amp, amp_off, mid, stats, ctl, lohi, partial,
        Ecol, Ncol, sums;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evk0 = nullptr, evk1 = nullptr, eve1 = nullptr;
    std::vector<hipEvent_t> chunk_ev;  // per-chunk timing and ordering of multi-chunk solves
    uint64_t generation = 0;          // bumped by every ma_build_system

    // captured launch sequence and the configuration it was captured for
    hipGraphExec_t gexec = nullptr;   // queue reset and the basis kernel
    hipGraphExec_t gexec1 = nullptr;  // the eigensolver kernel
    hipGraphExec_t gexec2 = nullptr;  // bisection, Fermi weighting, reductions
    hipGraphExec_t gexec0 = nullptr;  // descriptors and start network (learned start)
    std::vector<unsigned char> gkey;

    // caller-owned workspace (ma_set_workspace): the per-solve buffers are
    // carved from it instead of the library's own allocations
    char *user_ws = nullptr;
    size_t user_ws_bytes = 0;
    // allocation-free entry point: this device's static scratch
    void *scratch = nullptr;
    size_t scratch_bytes = 0;

    // The last solve that bisected the chemical potential: its Ritz data and
    // amplitudes stay where that solve wrote them, for ma_find_mu, until the
    // next solve, build or workspace change.
    bool last_valid = false;   // amplitudes of a bisected solve (ma_find_mu, ma_green)
    bool last_ritz = false;    // Ritz values and weights of the last solve (ma_dos)
    ma::DevSystem lastS{};
    ma::DevJob lastJ{};
    double *last_lohi = nullptr, *last_partial = nullptr, *last_sums = nullptr;

    // autotuned (slots per CU, schedule) per (p, q, precision)
    struct Tune { int p, q, prec, slots, sched, kernel, pipe; };
    std::vector<Tune> tunes;
    const Tune *find_tune(int p, int q, int prec) const
    {
        for (const auto &t : tunes)
            if (t.p == p && t.q == q && t.prec == prec) return &t;
        return nullptr;
    }
    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (gexec1) (void)hipGraphExecDestroy(gexec1);
        if (gexec2) (void)hipGraphExecDestroy(gexec2);
        if (gexec0) (void)hipGraphExecDestroy(gexec0);
        gexec = gexec1 = gexec2 = gexec0 = nullptr;
        gkey.clear();
    }

    ma_status fail(ma_status s, const char *fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return s;
    }
    ma_status hip_fail(hipError_t e, const char *what)
    {
        return fail(e == hipErrorOutOfMemory ? MA_ENOMEM : MA_EDEVICE, "%s: %s", what,
                    hipGetErrorString(e));
    }

    ma::DevSystem dev_system() const
    {
        ma::DevSystem S;
        S.o = o;
        S.n_atoms = n_atoms;
        S.nmax = nmax;
        S.maxpat = maxpat;
        S.blk_ptr = blk_ptr.as<int64_t>();
        S.blk_col = blk_col.as<int32_t>();
        S.Hd = Hd.as<double>();
        S.Sd = Sd.as<double>();
        S.Hf = Hf.as<float>();
        S.Sf = Sf.as<float>();
        S.reg_id = reg_id.as<int32_t>();
        S.reg_off = reg_off.as<int64_t>();
        S.reg_len = reg_len.as<int32_t>();
        S.lrp_off = lrp_off.as<int64_t>();
        S.lrp = lrp.as<int64_t>();
        S.lblk = lblk.as<int2>();
        S.jloc = jloc.as<int32_t>();
        S.blk_loc = blk_loc.as<int32_t>();
        S.out_loc = out_loc.as<int32_t>();
        S.max_nat = max_nat;
        S.max_lnnz = (int)max_lnnz;
        S.lidx = ma::global_lidx_fits(nmax, max_nat, (int)max_lnnz) ? 1 : 0;
        return S;
    }
};

#define HIPCHK(ctx, expr, what)                                 \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, what); \
    } while (0)

namespace {

// ---------------------------------------------------------------------------
// regions
// ---------------------------------------------------------------------------
struct CellGrid {
    bool periodic = false;
    double box[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, cs[3] = {1, 1, 1};
    int nc[3] = {1, 1, 1};
    std::vector<int32_t> start, atoms;   // atoms sorted by cell

    int cell_of(const double *x, int d) const
    {
        double f = (x[d] - lo[d]) / cs[d];
        int c = (int)std::floor(f);
        if (periodic) {
            c %= nc[d];
            if (c < 0) c += nc[d];
        } else {
            c = std::min(std::max(c, 0), nc[d] - 1);
        }
        return c;
    }
    void build(int n, const double *xyz, const double *bx, double cell_size)
    {
        periodic = bx != nullptr;
        for (int d = 0; d < 3; ++d) {
            double mn = 1e300, mx = -1e300;
            if (periodic) {
                mn = 0.0;
                mx = bx[d];
                box[d] = bx[d];
            } else {
                for (int a = 0; a < n; ++a) {
                    mn = std::min(mn, xyz[3 * a + d]);
                    mx = std::max(mx, xyz[3 * a + d]);
                }
                mx += 1e-9;
            }
            lo[d] = mn;
            nc[d] = std::max(1, std::min(512, (int)std::floor((mx - mn) / cell_size)));
            cs[d] = (mx - mn) / nc[d];
            if (cs[d] <= 0) cs[d] = 1.0;
        }
        const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
        std::vector<int64_t> cid(n);
        start.assign(ncell + 1, 0);
        for (int a = 0; a < n; ++a) {
            int64_t c = ((int64_t)cell_of(xyz + 3 * a, 0) * nc[1] + cell_of(xyz + 3 * a, 1)) * nc[2] +
                        cell_of(xyz + 3 * a, 2);
            cid[a] = c;
            start[c + 1]++;
        }
        for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
        atoms.assign(n, 0);
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int a = 0; a < n; ++a) atoms[fill[cid[a]]++] = a;
    }
};

inline double min_image_d2(const double *xyz, const double *box, int a, int b)
{
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double v = xyz[3 * b + k] - xyz[3 * a + k];
        if (box) v = v - box[k] * std::nearbyint(v / box[k]);
        d[k] = v;
    }
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

// Candidate atoms within squared distance r2 of atom a (all atoms if the
// search sphere covers the whole grid).  Appends (d2, atom).
void gather_within(const CellGrid &G, const double *xyz, const double *box, int n, int a, double r,
                   std::vector<std::pair<double, int32_t>> &out)
{
    out.clear();
    const double r2 = r * r;
    int span[3], c0[3];
    bool all = false;
    for (int d = 0; d < 3; ++d) {
        span[d] = (int)std::ceil(r / G.cs[d]);
        if (2 * span[d] + 1 >= G.nc[d]) all = true;
        c0[d] = G.cell_of(xyz + 3 * a, d);
    }
    if (all) {
        for (int b = 0; b < n; ++b) {
            double d2 = min_image_d2(xyz, box, a, b);
            if (d2 < r2) out.emplace_back(d2, b);
        }
        return;
    }
    for (int dx = -span[0]; dx <= span[0]; ++dx)
        for (int dy = -span[1]; dy <= span[1]; ++dy)
            for (int dz = -span[2]; dz <= span[2]; ++dz) {
                int c[3] = {c0[0] + dx, c0[1] + dy, c0[2] + dz};
                bool skip = false;
                for (int d = 0; d < 3; ++d) {
                    if (G.periodic) {
                        c[d] %= G.nc[d];
                        if (c[d] < 0) c[d] += G.nc[d];
                    } else if (c[d] < 0 || c[d] >= G.nc[d]) {
                        skip = true;
                    }
                }
                if (skip) continue;
                const int64_t cc = ((int64_t)c[0] * G.nc[1] + c[1]) * G.nc[2] + c[2];
                for (int32_t k = G.start[cc]; k < G.start[cc + 1]; ++k) {
                    const int b = G.atoms[k];
                    double d2 = min_image_d2(xyz, box, a, b);
                    if (d2 < r2) out.emplace_back(d2, b);
                }
            }
}

// Region atom lists (ascending): one shared list for MA_REGION_ALL, else one
// per atom.  Arguments are assumed validated.
void compute_regions(const ma_system *sys, const ma_region *reg,
                     std::vector<std::vector<int32_t>> &lists)
{
    const int n = sys->n_atoms;
    const bool shared = reg->mode == MA_REGION_ALL;
    lists.assign(shared ? 1 : n, {});
    if (shared) {
        lists[0].resize(n);
        std::iota(lists[0].begin(), lists[0].end(), 0);
    } else {
        const double *xyz = sys->xyz, *box = sys->box;
        double vol = 1.0;
        double lo3[3], hi3[3];
        for (int d = 0; d < 3; ++d) {
            lo3[d] = 1e300;
            hi3[d] = -1e300;
            for (int a = 0; a < n; ++a) {
                lo3[d] = std::min(lo3[d], xyz[3 * a + d]);
                hi3[d] = std::max(hi3[d], xyz[3 * a + d]);
            }
            vol *= box ? box[d] : std::max(1.0, hi3[d] - lo3[d]);
        }
        const double dens = n / vol;
        double rcell = reg->mode == MA_REGION_RADIUS ? reg->radius : 0.0;
        if (reg->mode == MA_REGION_NEAREST) {
            int kmax = 0;
            for (int a = 0; a < n; ++a) kmax = std::max(kmax, reg->n_rp_atom ? reg->n_rp_atom[a] : reg->n_rp);
            rcell = std::cbrt(3.0 * kmax / (4.0 * M_PI * dens));
        }
        CellGrid G;
        G.build(n, xyz, box, std::max(rcell, 1e-6) * 0.5);
        parallel_for(n, [&](int64_t a0, int64_t a1, int) {
            std::vector<std::pair<double, int32_t>> cand;
            for (int64_t a = a0; a < a1; ++a) {
                std::vector<int32_t> &L = lists[a];
                if (reg->mode == MA_REGION_RADIUS) {
                    gather_within(G, xyz, box, n, (int)a, reg->radius, cand);
                    // strict d2 < radius^2 as in gather_within
                    L.resize(cand.size());
                    for (size_t i = 0; i < cand.size(); ++i) L[i] = cand[i].second;
                } else {
                    const int k = reg->n_rp_atom ? reg->n_rp_atom[a] : reg->n_rp;
                    double r = std::cbrt(3.0 * k / (4.0 * M_PI * dens)) * 1.3 + 1e-9;
                    for (;;) {
                        gather_within(G, xyz, box, n, (int)a, r, cand);
                        if ((int)cand.size() >= k) break;
                        r *= 1.25;
                    }
                    std::partial_sort(cand.begin(), cand.begin() + k, cand.end());  // (d2, atom) order
                    L.resize(k);
                    for (int i = 0; i < k; ++i) L[i] = cand[i].second;
                }
                std::sort(L.begin(), L.end());
            }
        });
    }

}

// Validation of the region arguments shared by the entry points.
const char *check_region(const ma_system *sys, const ma_region *reg)
{
    const int n = sys->n_atoms;
    if (reg->mode != MA_REGION_ALL && reg->mode != MA_REGION_RADIUS && reg->mode != MA_REGION_NEAREST)
        return "unknown region mode";
    if (reg->mode != MA_REGION_ALL && !sys->xyz)
        return "positions are required for radius or nearest regions";
    if (sys->box)
        for (int d = 0; d < 3; ++d)
            if (!(sys->box[d] > 0)) return "box lengths must be positive";
    if (reg->mode == MA_REGION_RADIUS && !(reg->radius > 0)) return "region radius must be positive";
    if (reg->mode == MA_REGION_NEAREST)
        for (int a = 0; a < n; ++a) {
            const int k = reg->n_rp_atom ? reg->n_rp_atom[a] : reg->n_rp;
            if (k < 1 || k > n) return "n_rp out of range";
        }
    return nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
// public interface
// ---------------------------------------------------------------------------
extern "C" {

MA_API const char *ma_version(void) { return "marnoldi 0.1 (gfx950)"; }

MA_API void ma_default_opts(ma_opts *o)
{
    if (!o) return;
    o->precision = MA_PREC_FP64;
    o->cg_tol = 1e-12;
    o->inner_tol = 1e-6;
    o->max_refine = 8;
    o->breakdown_tau = 1e-10;
    o->spin = 2.0;
    o->n_target = NAN;
    o->start = MA_START_ZERO;
    o->slots_per_cu = 0;
    o->schedule = -1;
    o->use_graph = 1;
    o->basis_kernel = MA_BASIS_AUTO;
    o->chunk_columns = 0;
    o->pipeline = -1;
    o->keep_sj = 0;
}

MA_API ma_status ma_create(ma_ctx **out, int32_t device, void *stream)
{
    if (!out) return MA_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MA_EDEVICE;
    ma_ctx *c = new (std::nothrow) ma_ctx;
    if (!c) return MA_ENOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    if (hipSetDevice(device) != hipSuccess ||
        hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->evk0) != hipSuccess || hipEventCreate(&c->evk1) != hipSuccess ||
        hipEventCreate(&c->eve1) != hipSuccess ||
        hipEventCreateWithFlags(&c->evu, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->aux2, hipStreamNonBlocking) != hipSuccess ||
        ma::scratch_address(device, &c->scratch, &c->scratch_bytes) != hipSuccess) {
        delete c;
        return MA_EDEVICE;
    }
    *out = c;
    return MA_OK;
}

MA_API ma_status ma_destroy(ma_ctx *ctx)
{
    if (!ctx) return MA_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->evk0) (void)hipEventDestroy(ctx->evk0);
    if (ctx->evk1) (void)hipEventDestroy(ctx->evk1);
    if (ctx->eve1) (void)hipEventDestroy(ctx->eve1);
    for (hipEvent_t e : ctx->chunk_ev) (void)hipEventDestroy(e);
    ctx->chunk_ev.clear();
    ctx->drop_graph();
    if (ctx->evu) (void)hipEventDestroy(ctx->evu);
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->aux2) (void)hipStreamDestroy(ctx->aux2);
    delete ctx;
    return MA_OK;
}

MA_API const char *ma_last_error(const ma_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

MA_API ma_status ma_system_info(const ma_ctx *ctx, int64_t *M, int64_t *nblk, int32_t *nmax,
                                int32_t *maxpat)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->built) return MA_ESTATE;
    if (M) *M = ctx->M;
    if (nblk) *nblk = ctx->nblk;
    if (nmax) *nmax = ctx->nmax;
    if (maxpat) *maxpat = ctx->maxpat;
    return MA_OK;
}

// Place of every atom in Morton (Z-order) order of cells of edge two mean
// atomic spacings, ties by index; the index order without positions.  Atoms
// that are close in this order are close in space, so workgroups that run
// them at the same time share much of their region operators in the caches.
void spatial_order(int n, const double *xyz, const double *box, std::vector<int32_t> &rank)
{
    rank.resize(n);
    std::vector<int32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    if (xyz) {
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = box ? 0.0 : xyz[d];
            hi[d] = box ? box[d] : xyz[d];
        }
        auto coord = [&](int a, int d) {
            double v = xyz[3 * a + d];
            if (box) v -= box[d] * std::floor(v / box[d]);
            return v;
        };
        if (!box)
            for (int a = 0; a < n; ++a)
                for (int d = 0; d < 3; ++d) {
                    lo[d] = std::min(lo[d], xyz[3 * a + d]);
                    hi[d] = std::max(hi[d], xyz[3 * a + d]);
                }
        const double vol = std::max(1e-30, (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]));
        const double h = std::max(1e-12, 2.0 * std::cbrt(vol / n));
        std::vector<uint64_t> code(n, 0);
        for (int a = 0; a < n; ++a) {
            uint64_t c = 0;
            for (int d = 0; d < 3; ++d) {
                const double x = (coord(a, d) - lo[d]) / h;
                const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(x)));
                for (int b = 0; b < 21; ++b) c |= ((q >> b) & 1u) << (3 * b + d);
            }
            code[a] = c;
        }
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return code[x] < code[y]; });
    }
    for (int i = 0; i < n; ++i) rank[idx[i]] = i;
}

MA_API ma_status ma_build_system(ma_ctx *ctx, const ma_system *sys, const ma_region *reg)
{
    if (!ctx) return MA_EINVAL;
    if (!sys || !reg) return ctx->fail(MA_EINVAL, "null system or region");
    ctx->built = false;
    ctx->last_valid = ctx->last_ritz = false;
    ctx->drop_graph();
    ctx->generation++;
    const int n = sys->n_atoms, o = sys->n_orb;
    if (n < 1) return ctx->fail(MA_EINVAL, "n_atoms must be >= 1");
    if (o < 1 || o > MA_MAX_ORB) return ctx->fail(MA_EINVAL, "n_orb must be in 1..%d", MA_MAX_ORB);
    if (!sys->blk_ptr || !sys->blk_col || !sys->H || !sys->S)
        return ctx->fail(MA_EINVAL, "null matrix array");
    const int64_t *bp = sys->blk_ptr;
    const int32_t *bc = sys->blk_col;
    if (bp[0] != 0) return ctx->fail(MA_EINVAL, "blk_ptr[0] must be 0");
    for (int a = 0; a < n; ++a)
        if (bp[a + 1] < bp[a]) return ctx->fail(MA_EINVAL, "blk_ptr not monotone at atom %d", a);
    const int64_t nblk = bp[n];
    if (nblk > INT_MAX) return ctx->fail(MA_EINVAL, "more than 2^31 blocks");
    const int oo = o * o;
    // pattern: ascending columns in range, diagonal present
    for (int a = 0; a < n; ++a) {
        bool diag = false;
        for (int64_t k = bp[a]; k < bp[a + 1]; ++k) {
            if (bc[k] < 0 || bc[k] >= n) return ctx->fail(MA_EINVAL, "blk_col out of range in row %d", a);
            if (k > bp[a] && bc[k] <= bc[k - 1])
                return ctx->fail(MA_EINVAL, "blk_col not strictly ascending in row %d", a);
            if (bc[k] == a) diag = true;
        }
        if (!diag) return ctx->fail(MA_EINVAL, "diagonal block missing in row %d", a);
    }
    // values finite, pattern and values symmetric
    std::atomic<int64_t> bad(-1);
    std::atomic<int> bad_kind(0);
    parallel_for(n, [&](int64_t a0, int64_t a1, int) {
        for (int64_t a = a0; a < a1; ++a)
            for (int64_t k = bp[a]; k < bp[a + 1]; ++k) {
                for (int e = 0; e < oo; ++e)
                    if (!std::isfinite(sys->H[k * oo + e]) || !std::isfinite(sys->S[k * oo + e])) {
                        bad = a;
                        bad_kind = 1;
                        return;
                    }
                const int b = bc[k];
                const int32_t *lo = bc + bp[b], *hi = bc + bp[b + 1];
                const int32_t *f = std::lower_bound(lo, hi, (int32_t)a);
                if (f == hi || *f != a) {
                    bad = a;
                    bad_kind = 2;
                    return;
                }
                const int64_t kt = f - bc;
                for (int r = 0; r < o; ++r)
                    for (int c = 0; c < o; ++c) {
                        const double h1 = sys->H[k * oo + r * o + c], h2 = sys->H[kt * oo + c * o + r];
                        const double s1 = sys->S[k * oo + r * o + c], s2 = sys->S[kt * oo + c * o + r];
                        if (std::fabs(h1 - h2) > 1e-12 * std::max(1.0, std::fabs(h1)) ||
                            std::fabs(s1 - s2) > 1e-12 * std::max(1.0, std::fabs(s1))) {
                            bad = a;
                            bad_kind = 3;
                            return;
                        }
                    }
            }
    });
    if (bad >= 0) {
        static const char *what[] = {"", "non-finite value", "asymmetric block pattern",
                                     "asymmetric H or S values"};
        return ctx->fail(MA_EINVAL, "%s in block-row %lld", what[bad_kind.load()], (long long)bad.load());
    }

    // ---- regions ----
    if (const char *why = check_region(sys, reg)) return ctx->fail(MA_EINVAL, "%s", why);
    const bool shared = reg->mode == MA_REGION_ALL;
    const int nreg = shared ? 1 : n;
    std::vector<std::vector<int32_t>> lists;
    compute_regions(sys, reg, lists);
    // ---- local block index per region, pattern check ----
    std::vector<int32_t> h_reg_id(n), h_reg_len(nreg), h_jloc(n), h_blk_loc(nblk);
    std::vector<int64_t> h_reg_off(nreg + 1), h_lrp_off(nreg + 1), cnt(nreg + 1, 0);
    h_reg_off[0] = 0;
    for (int r = 0; r < nreg; ++r) {
        h_reg_len[r] = (int32_t)lists[r].size();
        h_reg_off[r + 1] = h_reg_off[r] + h_reg_len[r];
    }
    for (int a = 0; a < n; ++a) h_reg_id[a] = shared ? 0 : a;
    h_lrp_off[0] = 0;
    for (int r = 0; r < nreg; ++r) h_lrp_off[r + 1] = h_lrp_off[r] + h_reg_len[r] + 1;
    std::vector<int32_t> h_reg_atoms(h_reg_off[nreg]);
    for (int r = 0; r < nreg; ++r)
        std::copy(lists[r].begin(), lists[r].end(), h_reg_atoms.begin() + h_reg_off[r]);
    // count local blocks per region
    const unsigned nthr = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<std::vector<int32_t>> locs(nthr, std::vector<int32_t>(n, -1));
    parallel_for(nreg, [&](int64_t r0, int64_t r1, int t) {
        std::vector<int32_t> &loc = locs[t];
        for (int64_t r = r0; r < r1; ++r) {
            const auto &L = lists[r];
            for (size_t i = 0; i < L.size(); ++i) loc[L[i]] = (int32_t)i;
            int64_t c = 0;
            for (int32_t b : L)
                for (int64_t k = bp[b]; k < bp[b + 1]; ++k)
                    if (loc[bc[k]] >= 0) ++c;
            cnt[r + 1] = c;
            for (int32_t b : L) loc[b] = -1;
        }
    });
    std::vector<int64_t> lblk_off(nreg + 1, 0);
    for (int r = 0; r < nreg; ++r) lblk_off[r + 1] = lblk_off[r] + cnt[r + 1];
    std::vector<int64_t> h_lrp(h_lrp_off[nreg]);
    std::vector<int2> h_lblk(std::max<int64_t>(1, lblk_off[nreg]));
    std::atomic<int64_t> bad_region(-1);
    parallel_for(nreg, [&](int64_t r0, int64_t r1, int t) {
        std::vector<int32_t> &loc = locs[t];
        for (int64_t r = r0; r < r1; ++r) {
            const auto &L = lists[r];
            for (size_t i = 0; i < L.size(); ++i) loc[L[i]] = (int32_t)i;
            int64_t cur = lblk_off[r];
            int64_t *rp = h_lrp.data() + h_lrp_off[r];
            for (size_t i = 0; i < L.size(); ++i) {
                rp[i] = cur;
                const int32_t b = L[i];
                for (int64_t k = bp[b]; k < bp[b + 1]; ++k) {
                    const int32_t lc = loc[bc[k]];
                    if (lc >= 0) h_lblk[cur++] = make_int2(lc, (int)k);
                }
            }
            rp[L.size()] = cur;
            // atoms served by this region: all (shared) or atom r
            const int a0 = shared ? 0 : (int)r, a1 = shared ? n : (int)r + 1;
            for (int a = a0; a < a1; ++a) {
                if (loc[a] < 0) bad_region = a;
                h_jloc[a] = loc[a];
                for (int64_t k = bp[a]; k < bp[a + 1]; ++k) {
                    h_blk_loc[k] = loc[bc[k]];
                    if (loc[bc[k]] < 0) bad_region = a;
                }
            }
            for (int32_t b : L) loc[b] = -1;
        }
    });
    if (bad_region >= 0)
        return ctx->fail(MA_EINVAL, "region of atom %lld does not contain its block-row pattern",
                         (long long)bad_region.load());
    int nmax = 0, maxpat = 0, max_nat = 0;
    for (int r = 0; r < nreg; ++r) nmax = std::max(nmax, h_reg_len[r] * o);
    for (int r = 0; r < nreg; ++r) max_nat = std::max(max_nat, h_reg_len[r]);
    for (int a = 0; a < n; ++a) maxpat = std::max(maxpat, (int)(bp[a + 1] - bp[a]) * o);
    if (nmax > 8 * ma::kThreads)
        return ctx->fail(MA_EINVAL, "region dimension %d exceeds the supported %d", nmax,
                         8 * ma::kThreads);

    // ---- neighbour descriptors for the start network ----
    // For each atom: its kNbDesc nearest other atoms (by squared minimum-image
    // distance, then index) as (|d|/5, d/|d|), and the local positions, in its
    // own region, of its kNbOut nearest atoms (itself first).
    std::vector<float> h_geo;
    std::vector<int32_t> h_out_loc;
    const bool have_geo = sys->xyz != nullptr;
    if (have_geo) {
        const double *xyz = sys->xyz, *box = sys->box;
        h_geo.assign((size_t)n * ma::kGeoFeat, 0.0f);
        h_out_loc.assign((size_t)n * ma::kNbOut, -1);
        double lo3[3], hi3[3], vol = 1.0;
        for (int d = 0; d < 3; ++d) {
            lo3[d] = 1e300;
            hi3[d] = -1e300;
            for (int a = 0; a < n; ++a) {
                lo3[d] = std::min(lo3[d], xyz[3 * a + d]);
                hi3[d] = std::max(hi3[d], xyz[3 * a + d]);
            }
            vol *= box ? box[d] : std::max(1.0, hi3[d] - lo3[d]);
        }
        const int want = std::min(n, ma::kNbDesc + 1);
        const double r0 = std::cbrt(3.0 * want / (4.0 * M_PI * (n / vol))) * 1.3 + 1e-9;
        CellGrid G;
        G.build(n, xyz, box, r0 * 0.5);
        parallel_for(n, [&](int64_t a0, int64_t a1, int t) {
            std::vector<std::pair<double, int32_t>> cand;
            std::vector<int32_t> &loc = locs[t];
            for (int64_t a = a0; a < a1; ++a) {
                double r = r0;
                for (;;) {
                    gather_within(G, xyz, box, n, (int)a, r, cand);
                    if ((int)cand.size() >= want) break;
                    r *= 1.25;
                }
                std::partial_sort(cand.begin(), cand.begin() + want, cand.end());
                // rank 0 is the atom itself (distance 0)
                for (int k = 1; k < want && k <= ma::kNbDesc; ++k) {
                    const int b = cand[k].second;
                    double dv[3];
                    for (int d = 0; d < 3; ++d) {
                        double v = xyz[3 * b + d] - xyz[3 * a + d];
                        if (box) v = v - box[d] * std::nearbyint(v / box[d]);
                        dv[d] = v;
                    }
                    const double dist = std::sqrt(cand[k].first);
                    float *f = h_geo.data() + (size_t)a * ma::kGeoFeat + 4 * (k - 1);
                    f[0] = (float)(dist / 5.0);
                    for (int d = 0; d < 3; ++d) f[1 + d] = dist > 0 ? (float)(dv[d] / dist) : 0.0f;
                }
                const auto &L = lists[shared ? 0 : a];
                for (size_t i = 0; i < L.size(); ++i) loc[L[i]] = (int32_t)i;
                for (int k = 0; k < ma::kNbOut && k < want; ++k)
                    h_out_loc[(size_t)a * ma::kNbOut + k] = loc[cand[k].second];
                for (int32_t b : L) loc[b] = -1;
            }
        });
    }

    // transpose map of the block pattern: block (A, B) -> block (B, A)
    std::vector<int32_t> h_blk_t(nblk);
    parallel_for(n, [&](int64_t a0, int64_t a1, int) {
        for (int64_t a = a0; a < a1; ++a)
            for (int64_t k = bp[a]; k < bp[a + 1]; ++k) {
                const int b = bc[k];
                const int32_t *q = std::lower_bound(bc + bp[b], bc + bp[b + 1], (int32_t)a);
                h_blk_t[k] = (int32_t)(q - bc);
            }
    });

    // ---- upload ----
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    std::vector<float> Hf(nblk * oo), Sf(nblk * oo);
    for (int64_t e = 0; e < nblk * oo; ++e) {
        Hf[e] = (float)sys->H[e];
        Sf[e] = (float)sys->S[e];
    }
    auto up = [&](DevBuf &b, const void *src, size_t bytes, const char *what) -> ma_status {
        hipError_t e = b.reserve(bytes);
        if (e != hipSuccess) return ctx->hip_fail(e, what);
        if (bytes) {
            e = hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, ctx->stream);
            if (e != hipSuccess) return ctx->hip_fail(e, what);
        }
        return MA_OK;
    };
    ma_status s;
#define UP(buf, vec, what)                                                              \
    if ((s = up(ctx->buf, (vec), sizeof(*(vec)) * (size_t)(count_), what)) != MA_OK) return s;
    int64_t count_;
    count_ = n + 1;       UP(blk_ptr, bp, "blk_ptr")
    count_ = nblk;        UP(blk_col, bc, "blk_col")
    count_ = nblk * oo;   UP(Hd, sys->H, "H")
    count_ = nblk * oo;   UP(Sd, sys->S, "S")
    count_ = nblk * oo;   UP(Hf, Hf.data(), "H fp32")
    count_ = nblk * oo;   UP(Sf, Sf.data(), "S fp32")
    count_ = n;           UP(reg_id, h_reg_id.data(), "reg_id")
    count_ = nreg + 1;    UP(reg_off, h_reg_off.data(), "reg_off")
    count_ = nreg;        UP(reg_len, h_reg_len.data(), "reg_len")
    count_ = nreg + 1;    UP(lrp_off, h_lrp_off.data(), "lrp_off")
    count_ = (int64_t)h_lrp.size();  UP(lrp, h_lrp.data(), "lrp")
    count_ = (int64_t)h_lblk.size(); UP(lblk, h_lblk.data(), "lblk")
    count_ = n;           UP(jloc, h_jloc.data(), "jloc")
    count_ = nblk;        UP(blk_loc, h_blk_loc.data(), "blk_loc")
    count_ = nblk;        UP(blk_t, h_blk_t.data(), "blk_t")
    count_ = (int64_t)h_reg_atoms.size(); UP(reg_atoms, h_reg_atoms.data(), "reg_atoms")
    if (have_geo) {
        count_ = (int64_t)h_geo.size();     UP(geo, h_geo.data(), "descriptors")
        count_ = (int64_t)h_out_loc.size(); UP(out_loc, h_out_loc.data(), "neighbours")
    }
#undef UP
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "upload");
    ctx->have_geo = have_geo;
    if (ctx->net.ready && ctx->o != o) ctx->net.ready = false;   // shape changed
    ctx->o = o;
    ctx->n_atoms = n;
    ctx->nblk = nblk;
    ctx->M = (int64_t)n * o;
    ctx->nmax = nmax;
    ctx->maxpat = maxpat;
    ctx->max_nat = max_nat;
    ctx->nreg = nreg;
    ctx->reg_atoms_total = (int64_t)h_reg_atoms.size();
    ctx->max_lnnz = 0;
    for (int r = 0; r < nreg; ++r) ctx->max_lnnz = std::max<int64_t>(ctx->max_lnnz, cnt[r + 1]);
    ctx->reg_len_of_atom.resize(n);
    ctx->lblk_of_atom.resize(n);
    ctx->pat_blocks.resize(n);
    for (int a = 0; a < n; ++a) {
        ctx->reg_len_of_atom[a] = h_reg_len[h_reg_id[a]];
        ctx->lblk_of_atom[a] = cnt[h_reg_id[a] + 1];
        ctx->pat_blocks[a] = (int32_t)(bp[a + 1] - bp[a]);
    }
    spatial_order(n, sys->xyz, sys->box, ctx->spatial_rank);
    ctx->built = true;
    return MA_OK;
}

MA_API ma_status ma_region_sizes(const ma_ctx *ctx, int32_t *region_atoms, int64_t *local_blocks)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->built) return MA_ESTATE;
    if (region_atoms) std::copy(ctx->reg_len_of_atom.begin(), ctx->reg_len_of_atom.end(), region_atoms);
    if (local_blocks) std::copy(ctx->lblk_of_atom.begin(), ctx->lblk_of_atom.end(), local_blocks);
    return MA_OK;
}

MA_API int64_t ma_region_atoms(const ma_system *sys, const ma_region *reg, int32_t atom,
                                int32_t *out, int64_t cap)
{
    if (!sys || !reg || sys->n_atoms < 1 || atom < 0 || atom >= sys->n_atoms) return MA_EINVAL;
    if (check_region(sys, reg)) return MA_EINVAL;
    ma_system one = *sys;
    std::vector<std::vector<int32_t>> lists;
    if (reg->mode == MA_REGION_ALL) {
        compute_regions(&one, reg, lists);
    } else {
        // the same construction, restricted to one atom
        std::vector<std::vector<int32_t>> all;
        compute_regions(&one, reg, all);
        lists.assign(1, std::move(all[atom]));
    }
    const auto &L = lists[0];
    for (int64_t i = 0; i < (int64_t)L.size() && i < cap; ++i) out[i] = L[i];
    return (int64_t)L.size();
}

}  // extern "C"

namespace {

// Everything one launch sequence needs, resolved from the arguments.
struct Plan {
    ma_opts opts;
    int p = 0, q = 0, nu = 0, slots = 0, sched = 0;
    double mu = 0, kT = 0, n_target = 0;
    bool bisect = false;
    int kind = ma::kBasisWorkspace;   // basis kernel
    int nchunks = 0, max_cn = 0;      // chunks of the processing order
    bool pipelined = false;           // eigensolver of chunk k on the aux stream
    int nbuf = 1;                     // chunk buffers in the ring (pipelined: >= 2)
    std::vector<int32_t> ch_c0, ch_cn, ch_items;   // per chunk: first column position,
                                                   // columns, work items
    std::vector<int32_t> hcols;
    ma::DevSystem S;
    ma::DevJob J;                // J.c0, J.cn, J.qbounds describe chunk 0
    const int32_t *qb_dev = nullptr;
    double *rho = nullptr, *pi = nullptr;
    // per-solve device buffers (the library's own, or carved from a caller
    // workspace or the allocation-free scratch)
    float *feat = nullptr, *x0 = nullptr;
    int *ctl = nullptr;
    double *lohi = nullptr, *partial = nullptr, *sums = nullptr;
    size_t bytes = 0;              // bytes the buffers take (sizing)
    bool timed_chunks = true;      // per-chunk timing events (multi-chunk solves)
    ma::DevJob chunk_job(int k) const
    {
        ma::DevJob Jk = J;
        Jk.c0 = ch_c0[k];
        Jk.cn = ch_cn[k];
        Jk.qbounds = qb_dev + (int64_t)k * (J.nqueues + 1);
        // pipelined: chunk k uses buffer k mod nbuf of the ring
        if (nbuf > 1) Jk.mid = J.mid + (int64_t)(k % nbuf) * max_cn * J.mid_stride;
        return Jk;
    }
};

// Chunk buffer budget: the Galerkin pairs and basis rows of the columns of
// one chunk (the rest of the solve's memory is proportional to the system);
// a pipelined solve keeps a ring of such buffers within kRingBudget, so the
// basis kernel of chunk k waits only for the eigensolver of chunk k - nbuf.
// Unpipelined solves on the library's own buffers take a fifth of the device
// memory that is free (counting the chunk buffer they already hold), between
// 4 and 64 GiB: fewer, longer chunks lose less to each chunk's drain (on the
// 262,144-atom cell 60 chunks of 4 GiB cost 4.6 % over 4 of 65 GB); a
// caller's workspace and size queries keep 4 GiB so that the two agree.
constexpr size_t kMidBudget = (size_t)4 << 30;
constexpr size_t kMidBudgetMax = (size_t)64 << 30;
constexpr size_t kRingBudget = (size_t)8 << 30;

// Where the per-solve buffers of a plan come from: the library's own
// allocations (grown as needed), or consecutive 256-byte aligned pieces of a
// caller-provided region (a caller workspace, or the allocation-free
// scratch); with `size_only` nothing is placed and only the bytes are counted.
struct BufSource {
    char *base = nullptr;      // null: the library's own allocations
    size_t cap = 0;
    size_t off = 0;
    bool size_only = false;
    bool limited = false;      // the region is small: cap the chunk buffer and
                               // the persistent workgroups to fit
    bool region() const { return base != nullptr || size_only; }
    void *take(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        void *ptr = size_only ? nullptr : base + off;
        off += n;
        return ptr;
    }
};

ma_status make_plan(ma_ctx *ctx, int64_t ncols, const int32_t *cols, int32_t p, int32_t q,
                    double mu, double kT, const ma_opts *opts_in, double *rho, double *pi,
                    double *eps, double *wts, int32_t *col_stats, float *sj_near,
                    int slots_override, int sched_override, Plan &P, BufSource *src = nullptr)
{
    BufSource own;
    if (!src) src = &own;
    if (!ctx->built) return ctx->fail(MA_ESTATE, "ma_build_system has not succeeded");
    ma_default_opts(&P.opts);
    if (opts_in) P.opts = *opts_in;
    const ma_opts &opts = P.opts;
    if (p < 1 || q < 0 || p + q > MA_MAX_NU)
        return ctx->fail(MA_EINVAL, "need p >= 1, q >= 0, p + q <= %d", MA_MAX_NU);
    if (!(kT > 0) || !std::isfinite(kT)) return ctx->fail(MA_EINVAL, "kT must be positive");
    if (std::isinf(mu)) return ctx->fail(MA_EINVAL, "mu must be finite or NaN");
    if (opts.precision != MA_PREC_FP64 && opts.precision != MA_PREC_MIXED &&
        opts.precision != MA_PREC_MIXED_F64ACC)
        return ctx->fail(MA_EINVAL, "unknown precision %d", opts.precision);
    if (!(opts.cg_tol > 0) || !(opts.breakdown_tau >= 0) || !(opts.inner_tol > 0) || opts.max_refine < 0)
        return ctx->fail(MA_EINVAL, "invalid tolerances");
    if (opts.start != MA_START_ZERO && opts.start != MA_START_LEARNED &&
        opts.start != MA_START_PREVIOUS)
        return ctx->fail(MA_EINVAL, "unknown start %d", opts.start);
    if (opts.start == MA_START_PREVIOUS &&
        !(ctx->sj_valid && ctx->sj_n_atoms == ctx->n_atoms && ctx->sj_o == ctx->o))
        return ctx->fail(MA_EINVAL, "the previous start needs s_j kept (keep_sj) by a solve on "
                         "the same atoms");
    if (opts.keep_sj != 0 && opts.keep_sj != 1) return ctx->fail(MA_EINVAL, "keep_sj must be 0 or 1");
    if (opts.start == MA_START_LEARNED && !(ctx->net.ready && ctx->have_geo))
        return ctx->fail(MA_EINVAL, "learned start needs a start model and positions");
    if (opts.schedule < -1 || opts.schedule > MA_SCHED_SPATIAL)
        return ctx->fail(MA_EINVAL, "unknown schedule %d", opts.schedule);
    if (cols == nullptr) ncols = ctx->M;
    if (ncols < 1 || ncols > INT_MAX) return ctx->fail(MA_EINVAL, "ncols out of range");
    P.hcols.resize(ncols);
    for (int64_t c = 0; c < ncols; ++c) {
        P.hcols[c] = cols ? cols[c] : (int32_t)c;
        if (P.hcols[c] < 0 || P.hcols[c] >= ctx->M)
            return ctx->fail(MA_EINVAL, "column %lld out of range", (long long)P.hcols[c]);
    }
    P.p = p;
    P.q = q;
    P.nu = p + q;
    P.mu = mu;
    P.kT = kT;
    P.bisect = std::isnan(mu);
    P.n_target = std::isnan(opts.n_target) ? 0.5 * (double)ncols : opts.n_target;
    P.rho = rho;
    P.pi = pi;
    if (sj_near && !ctx->have_geo) return ctx->fail(MA_EINVAL, "sj_near needs positions");

    // launch configuration: explicit, autotuned, or defaults
    const ma_ctx::Tune *tn = ctx->find_tune(p, q, opts.precision);
    P.sched = sched_override >= 0 ? sched_override
              : opts.schedule >= 0 ? opts.schedule : (tn ? tn->sched : MA_SCHED_LPT);
    const int pipe = opts.pipeline >= 0 ? opts.pipeline : (tn && tn->pipe >= 0 ? tn->pipe : 4);

    ma::DevSystem &S = P.S;
    ma::DevJob &J = P.J;
    S = ctx->dev_system();
    std::memset(&J, 0, sizeof J);   // the launch key compares the raw bytes
    J.ncols = (int)ncols;
    J.p = p;
    J.q = q;
    J.nu = P.nu;
    J.precision = opts.precision;
    J.cg_tol = opts.cg_tol;
    J.inner_tol = opts.inner_tol;
    J.tau = opts.breakdown_tau;
    J.max_refine = opts.max_refine;
    if (opts.basis_kernel < MA_BASIS_AUTO || opts.basis_kernel > MA_BASIS_ATOM)
        return ctx->fail(MA_EINVAL, "unknown basis kernel %d", opts.basis_kernel);
    if (opts.chunk_columns < 0) return ctx->fail(MA_EINVAL, "chunk_columns must be >= 0");
    if (opts.pipeline < -1) return ctx->fail(MA_EINVAL, "pipeline must be >= -1");
    const bool fits = ma::basis_small_fits(ctx->nmax, P.nu, q, ctx->o);
    const bool gfits = ma::basis_group_fits(ctx->nmax, P.nu, ctx->o);
    const bool afits = ma::basis_atom_fits(ctx->nmax, P.nu, ctx->o, opts.precision);
    if (opts.basis_kernel == MA_BASIS_ONCHIP && !fits)
        return ctx->fail(MA_EINVAL, "the on-chip basis kernel cannot hold regions of %d orbitals "
                         "with p = %d, q = %d", ctx->nmax, p, q);
    if (opts.basis_kernel == MA_BASIS_GROUP && !gfits)
        return ctx->fail(MA_EINVAL, "the atom-group basis kernel needs 4 or 9 orbitals per atom "
                         "and regions it can stage (o = %d, %d orbitals)", ctx->o, ctx->nmax);
    if (opts.basis_kernel == MA_BASIS_ATOM && !afits)
        return ctx->fail(MA_EINVAL, "the atom basis kernel needs 4 or 9 orbitals per atom, an "
                         "FP64-vector precision mode and regions it can stage (o = %d, %d "
                         "orbitals, precision %d)", ctx->o, ctx->nmax, opts.precision);
    // automatic choice: the autotuned kernel if there is one, else the
    // workspace kernel (the fastest untuned choice on every shape measured)
    int want_kernel = opts.basis_kernel;
    if (want_kernel == MA_BASIS_AUTO)
        want_kernel = tn && tn->kernel != MA_BASIS_AUTO ? tn->kernel : MA_BASIS_WORKSPACE;
    // the group kernel neither starts from nor keeps whole-region s_j
    const bool sj_io = opts.start == MA_START_PREVIOUS || opts.keep_sj;
    if (opts.basis_kernel == MA_BASIS_GROUP && sj_io)
        return ctx->fail(MA_EINVAL, "the atom-group basis kernel does not keep or reuse s_j");
    if ((want_kernel == MA_BASIS_ONCHIP && !fits) || (want_kernel == MA_BASIS_GROUP && !gfits) ||
        (want_kernel == MA_BASIS_ATOM && !afits) || (want_kernel == MA_BASIS_GROUP && sj_io))
        want_kernel = MA_BASIS_WORKSPACE;
    P.kind = want_kernel == MA_BASIS_ONCHIP ? ma::kBasisOnchip
             : want_kernel == MA_BASIS_GROUP ? ma::kBasisGroup
             : want_kernel == MA_BASIS_ATOM ? ma::kBasisAtom : ma::kBasisWorkspace;
    const int o = ctx->o;
    J.lidx = P.kind == ma::kBasisWorkspace ? S.lidx
             : P.kind == ma::kBasisOnchip
                 ? (ma::onchip_lidx_fits(ctx->nmax, P.nu, ctx->max_nat, (int)ctx->max_lnnz) ? 1 : 0)
             : P.kind == ma::kBasisAtom
                 ? (ma::atom_lidx_fits(ctx->nmax, o, ctx->max_nat, (int)ctx->max_lnnz) ? 1 : 0)
                 : 0;
    J.ws_stride = P.kind == ma::kBasisOnchip ? 0
                  : P.kind == ma::kBasisAtom ? ma::atom_ws_doubles(o, P.nu, q, ctx->nmax)
                  : (int64_t)(P.kind == ma::kBasisGroup ? ma::basis_group_width(o) : 1) *
                        (3 * P.nu + q) * ctx->nmax;
    int bpc = 0;
    hipError_t e = ma::basis_occupancy(S, J, P.kind, &bpc);
    if (e != hipSuccess) return ctx->hip_fail(e, "occupancy");
    if (bpc < 1)
        return ctx->fail(MA_EINVAL, "basis kernel does not fit on a compute unit (nu=%d, nmax=%d)",
                         P.nu, ctx->nmax);
    int want = slots_override > 0 ? slots_override
               : opts.slots_per_cu > 0 ? opts.slots_per_cu : (tn ? tn->slots : bpc);
    bpc = std::min(bpc, std::max(1, want));

    // Work items: single columns, or (atom-group kernel) the requested
    // columns of one atom.  items[w] lists the output rows of item w.
    std::vector<int32_t> item_start, item_cols;
    if (P.kind == ma::kBasisGroup || P.kind == ma::kBasisAtom) {
        // the requested columns of each atom (atoms in order of first
        // appearance), cut into runs of at most the kernel's width
        const int width = P.kind == ma::kBasisAtom ? o : ma::basis_group_width(o);
        std::vector<int32_t> first(ctx->n_atoms, -1), count(ctx->n_atoms, 0);
        std::vector<int32_t> atoms;
        for (int64_t c = 0; c < ncols; ++c) {
            const int A = P.hcols[c] / o;
            if (first[A] < 0) {
                first[A] = (int32_t)atoms.size();
                atoms.push_back(A);
            }
            ++count[A];
        }
        std::vector<int32_t> astart(atoms.size() + 1, 0);
        for (size_t g = 0; g < atoms.size(); ++g) astart[g + 1] = astart[g] + count[atoms[g]];
        std::vector<int32_t> bycol(ncols), fill(atoms.size(), 0);
        for (int64_t c = 0; c < ncols; ++c) {
            const int g = first[P.hcols[c] / o];
            bycol[astart[g] + fill[g]++] = (int32_t)c;
        }
        item_cols = bycol;
        item_start.clear();
        for (size_t g = 0; g < atoms.size(); ++g)
            for (int32_t u = astart[g]; u < astart[g + 1]; u += width) item_start.push_back(u);
        item_start.push_back((int32_t)ncols);
    } else {
        item_start.resize(ncols + 1);
        std::iota(item_start.begin(), item_start.end(), 0);
        item_cols.resize(ncols);
        std::iota(item_cols.begin(), item_cols.end(), 0);
    }
    const int nitems = (int)item_start.size() - 1;
    auto item_len = [&](int w) { return item_start[w + 1] - item_start[w]; };
    auto item_region = [&](int w) { return ctx->reg_len_of_atom[P.hcols[item_cols[item_start[w]]] / o]; };
    auto item_atom = [&](int w) { return P.hcols[item_cols[item_start[w]]] / o; };

    // chunks: whole work items, at most the chunk budget of columns each
    J.mid_stride = ma::mid_stride_of(P.nu, ctx->maxpat);
    size_t mid_budget = src->limited ? src->cap / 4 : kMidBudget;
    if (!src->region() && pipe < 2) {   // (a pipelined ring keeps 4 GiB buffers)
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess)
            mid_budget = std::min(kMidBudgetMax, std::max(kMidBudget, (fr + ctx->mid.bytes) / 5));
    }
    const int64_t per_chunk = std::max<int64_t>(o, (int64_t)(mid_budget / (sizeof(double) * J.mid_stride)));
    int64_t budget = std::max<int64_t>(1, opts.chunk_columns > 0 ? opts.chunk_columns : per_chunk);
    // pipelining: for solves large enough, opts.pipeline + 2 chunks whose
    // sizes fall geometrically (ratio 0.75, the best of 0.6-0.8 measured), so
    // the eigensolver of each chunk fits beside the basis kernel of the next
    // and the last one, which nothing overlaps, is short; equal chunks where
    // the chunk buffer caps the first
    std::vector<int64_t> target;   // column target per chunk
    if (pipe >= 2 && ncols >= (int64_t)pipe * 2048) {
        const int nch = pipe + 2;
        const double r = 0.75;
        double norm = 0.0;
        for (int k = 0; k < nch; ++k) norm += std::pow(r, k);
        for (int k = 0; k < nch; ++k)
            target.push_back(std::max<int64_t>(1, std::llround((double)ncols * std::pow(r, k) / norm)));
        if (target[0] > budget) {
            target.clear();
            budget = std::min<int64_t>(budget, (ncols + pipe - 1) / pipe);
        }
    }
    std::vector<int32_t> ch_item0;   // first work item of each chunk
    {
        int64_t cols_in = 0;
        for (int w = 0; w < nitems; ++w) {
            const size_t k = ch_item0.size() - 1;   // current chunk (w > 0)
            const int64_t lim = (w > 0 && k < target.size()) ? target[k] : budget;
            if (w == 0 || cols_in + item_len(w) > lim) {
                ch_item0.push_back(w);
                cols_in = 0;
            }
            cols_in += item_len(w);
        }
        ch_item0.push_back(nitems);
    }
    P.nchunks = (int)ch_item0.size() - 1;
    P.pipelined = pipe >= 2 && P.nchunks >= 2;

    // processing order of the work items, per chunk and queue
    std::vector<int32_t> witem(nitems);
    std::iota(witem.begin(), witem.end(), 0);
    auto lpt = [&](std::vector<int32_t>::iterator b, std::vector<int32_t>::iterator e2) {
        std::stable_sort(b, e2, [&](int32_t x, int32_t y) { return item_region(x) > item_region(y); });
    };
    const bool xcd = P.sched == MA_SCHED_XCD_INPUT || P.sched == MA_SCHED_XCD_LPT;
    J.nqueues = xcd ? ma::kMaxQueues : 1;
    std::vector<int32_t> qb((size_t)P.nchunks * (J.nqueues + 1));
    P.ch_c0.assign(P.nchunks, 0);
    P.ch_cn.assign(P.nchunks, 0);
    P.ch_items.assign(P.nchunks, 0);
    for (int k = 0; k < P.nchunks; ++k) {
        const int w0 = ch_item0[k], w1 = ch_item0[k + 1], nw = w1 - w0;
        for (int i = 0; i <= J.nqueues; ++i)
            qb[(size_t)k * (J.nqueues + 1) + i] = (int32_t)(w0 + (int64_t)nw * i / J.nqueues);
        if (P.sched == MA_SCHED_LPT) lpt(witem.begin() + w0, witem.begin() + w1);
        if (P.sched == MA_SCHED_SPATIAL)
            std::stable_sort(witem.begin() + w0, witem.begin() + w1, [&](int32_t x, int32_t y) {
                return ctx->spatial_rank[item_atom(x)] < ctx->spatial_rank[item_atom(y)];
            });
        if (P.sched == MA_SCHED_XCD_LPT)
            for (int i = 0; i < J.nqueues; ++i)
                lpt(witem.begin() + qb[(size_t)k * (J.nqueues + 1) + i],
                    witem.begin() + qb[(size_t)k * (J.nqueues + 1) + i + 1]);
        P.ch_items[k] = nw;
    }
    // column order: the columns of the work items in processing order;
    // gstart[w] is the first column position of the w-th processed item
    std::vector<int32_t> order(ncols), gstart(nitems + 1, 0);
    {
        int32_t pos = 0;
        for (int w = 0; w < nitems; ++w) {
            gstart[w] = pos;
            const int it = witem[w];
            for (int u = item_start[it]; u < item_start[it + 1]; ++u) order[pos++] = item_cols[u];
        }
        gstart[nitems] = pos;
        for (int k = 0; k < P.nchunks; ++k) {
            P.ch_c0[k] = gstart[ch_item0[k]];
            P.ch_cn[k] = gstart[ch_item0[k + 1]] - gstart[ch_item0[k]];
            P.max_cn = std::max(P.max_cn, P.ch_cn[k]);
        }
    }
    if (P.pipelined) {
        const size_t buf = sizeof(double) * (size_t)J.mid_stride * std::max(1, P.max_cn);
        P.nbuf = (int)std::max<size_t>(2, std::min<size_t>((size_t)P.nchunks, kRingBudget / buf));
    } else {
        P.nbuf = 1;
    }
    int max_items = 0;
    for (int k = 0; k < P.nchunks; ++k) max_items = std::max(max_items, P.ch_items[k]);
    P.slots = (int)std::min<int64_t>((int64_t)bpc * ctx->cu_count, max_items);
    // amplitudes (only while the chemical potential is unknown), compact per column
    std::vector<int64_t> aoff;
    size_t amp_elems = 0;
    if (P.bisect) {
        aoff.resize(ncols + 1);
        aoff[0] = 0;
        for (int64_t c = 0; c < ncols; ++c) {
            const int A = P.hcols[c] / o;
            aoff[c + 1] = aoff[c] + (int64_t)ctx->pat_blocks[A] * o * P.nu;
        }
        amp_elems = (size_t)aoff[ncols];
    }
    const size_t amp_bytes = (opts.precision == MA_PREC_FP64 ? sizeof(double) : sizeof(float)) *
                             std::max<size_t>(1, amp_elems);

    // per-solve buffers: the library's own, or pieces of the caller's region
    const bool learned = opts.start == MA_START_LEARNED;
    const size_t n_cols = sizeof(int32_t) * ncols, n_order = sizeof(int32_t) * ncols,
                 n_qb = sizeof(int32_t) * qb.size(), n_gstart = sizeof(int32_t) * (nitems + 1),
                 n_eps = eps ? 0 : sizeof(double) * (size_t)ncols * P.nu,
                 n_wts = wts ? 0 : sizeof(double) * (size_t)ncols * P.nu,
                 n_amp = P.bisect ? amp_bytes : 0,
                 n_aoff = P.bisect ? sizeof(int64_t) * (ncols + 1) : 0,
                 n_stats = col_stats ? 0 : sizeof(int32_t) * (size_t)ncols * ma::kStats,
                 n_feat = learned ? sizeof(float) * (size_t)ncols * ctx->net.nf : 0,
                 n_x0 = learned ? sizeof(float) * (size_t)ncols * ctx->net.no : 0,
                 n_x0full = opts.start == MA_START_PREVIOUS
                                ? sizeof(double) * (size_t)ncols * ctx->nmax : 0,
                 n_ctl = sizeof(int) * 16, n_lohi = sizeof(double) * 2,
                 n_partial = sizeof(double) * (ma::kCountBlocks * ma::kBisectTrials + 1),
                 n_E = sizeof(double) * ncols, n_sums = sizeof(double) * 2,
                 n_mid = sizeof(double) * (size_t)J.mid_stride * P.max_cn * P.nbuf,
                 slot_bytes = P.kind == ma::kBasisOnchip ? 0 : sizeof(double) * (size_t)J.ws_stride;
    void *b_cols, *b_order, *b_qb, *b_gstart, *b_ws = nullptr, *b_mid, *b_eps = nullptr,
         *b_wts = nullptr, *b_amp = nullptr, *b_aoff = nullptr, *b_stats = nullptr,
         *b_feat = nullptr, *b_x0 = nullptr, *b_x0full = nullptr, *b_ctl, *b_lohi, *b_partial,
         *b_E, *b_N, *b_sums;
    if (src->region()) {
        b_cols = src->take(n_cols);
        b_order = src->take(n_order);
        b_qb = src->take(n_qb);
        b_gstart = src->take(n_gstart);
        b_mid = src->take(n_mid);
        if (n_eps) b_eps = src->take(n_eps);
        if (n_wts) b_wts = src->take(n_wts);
        if (n_amp) b_amp = src->take(n_amp);
        if (n_aoff) b_aoff = src->take(n_aoff);
        if (n_stats) b_stats = src->take(n_stats);
        if (n_feat) b_feat = src->take(n_feat);
        if (n_x0) b_x0 = src->take(n_x0);
        if (n_x0full) b_x0full = src->take(n_x0full);
        b_ctl = src->take(n_ctl);
        b_lohi = src->take(n_lohi);
        b_partial = src->take(n_partial);
        b_E = src->take(n_E);
        b_N = src->take(n_E);
        b_sums = src->take(n_sums);
        if (slot_bytes) {
            if (src->limited) {
                // as many persistent workgroups as the rest of the region holds
                const size_t used = (src->off + 255) & ~(size_t)255;
                const int64_t fit = used < src->cap ? (int64_t)((src->cap - used) / slot_bytes) : 0;
                if (fit < 1)
                    return ctx->fail(MA_EINVAL, "the solve needs more than the %zu-byte scratch "
                                     "(%zu bytes before the first basis workspace of %zu bytes)",
                                     src->cap, used, slot_bytes);
                P.slots = (int)std::min<int64_t>(P.slots, fit);
            }
            b_ws = src->take(slot_bytes * P.slots);
        }
        P.bytes = (src->off + 255) & ~(size_t)255;
        if (src->size_only) return MA_OK;
        if (src->off > src->cap)
            return ctx->fail(MA_EINVAL, "the solve needs %zu bytes of workspace, %zu given",
                             src->off, src->cap);
    } else {
        HIPCHK(ctx, ctx->cols.reserve(n_cols), "cols");
        HIPCHK(ctx, ctx->order.reserve(n_order), "order");
        HIPCHK(ctx, ctx->qbounds.reserve(n_qb), "queues");
        HIPCHK(ctx, ctx->gstart.reserve(n_gstart), "work items");
        if (slot_bytes) HIPCHK(ctx, ctx->ws.reserve(slot_bytes * P.slots), "workspace");
        HIPCHK(ctx, ctx->mid.reserve(n_mid), "chunk buffer");
        if (n_eps) HIPCHK(ctx, ctx->eps.reserve(n_eps), "eps");
        if (n_wts) HIPCHK(ctx, ctx->wts.reserve(n_wts), "wts");
        if (n_amp) HIPCHK(ctx, ctx->amp.reserve(n_amp), "amplitudes");
        if (n_aoff) HIPCHK(ctx, ctx->amp_off.reserve(n_aoff), "amplitude offsets");
        if (n_stats) HIPCHK(ctx, ctx->stats.reserve(n_stats), "stats");
        if (n_feat) HIPCHK(ctx, ctx->feat.reserve(n_feat), "descriptors");
        if (n_x0) HIPCHK(ctx, ctx->x0.reserve(n_x0), "start vectors");
        if (n_x0full) HIPCHK(ctx, ctx->x0full.reserve(n_x0full), "previous start vectors");
        HIPCHK(ctx, ctx->ctl.reserve(n_ctl), "ctl");
        HIPCHK(ctx, ctx->lohi.reserve(n_lohi), "lohi");
        HIPCHK(ctx, ctx->partial.reserve(n_partial), "partial");
        HIPCHK(ctx, ctx->Ecol.reserve(n_E), "Ecol");
        HIPCHK(ctx, ctx->Ncol.reserve(n_E), "Ncol");
        HIPCHK(ctx, ctx->sums.reserve(n_sums), "sums");
        b_cols = ctx->cols.p;
        b_order = ctx->order.p;
        b_qb = ctx->qbounds.p;
        b_gstart = ctx->gstart.p;
        b_ws = slot_bytes ? ctx->ws.p : nullptr;
        b_mid = ctx->mid.p;
        b_eps = n_eps ? ctx->eps.p : nullptr;
        b_wts = n_wts ? ctx->wts.p : nullptr;
        b_amp = n_amp ? ctx->amp.p : nullptr;
        b_aoff = n_aoff ? ctx->amp_off.p : nullptr;
        b_stats = n_stats ? ctx->stats.p : nullptr;
        b_feat = n_feat ? ctx->feat.p : nullptr;
        b_x0 = n_x0 ? ctx->x0.p : nullptr;
        b_x0full = n_x0full ? ctx->x0full.p : nullptr;
        b_ctl = ctx->ctl.p;
        b_lohi = ctx->lohi.p;
        b_partial = ctx->partial.p;
        b_E = ctx->Ecol.p;
        b_N = ctx->Ncol.p;
        b_sums = ctx->sums.p;
    }
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    HIPCHK(ctx, hipMemcpyAsync(b_cols, P.hcols.data(), n_cols, hipMemcpyHostToDevice, st), "cols");
    HIPCHK(ctx, hipMemcpyAsync(b_order, order.data(), n_order, hipMemcpyHostToDevice, st), "order");
    HIPCHK(ctx, hipMemcpyAsync(b_qb, qb.data(), n_qb, hipMemcpyHostToDevice, st), "queues");
    HIPCHK(ctx, hipMemcpyAsync(b_gstart, gstart.data(), n_gstart, hipMemcpyHostToDevice, st), "work items");
    if (P.bisect)
        HIPCHK(ctx, hipMemcpyAsync(b_aoff, aoff.data(), n_aoff, hipMemcpyHostToDevice, st), "amplitude offsets");
    // start vectors from the kept s_j (mapped onto the current regions)
    if (opts.start == MA_START_PREVIOUS) {
        ma::RegionView cur{ctx->reg_id.as<int32_t>(), ctx->reg_len.as<int32_t>(),
                           ctx->reg_atoms.as<int32_t>(), ctx->reg_off.as<int64_t>(), ctx->nmax};
        ma::RegionView old{ctx->sj_reg_id.as<int32_t>(), ctx->sj_reg_len.as<int32_t>(),
                           ctx->sj_reg_atoms.as<int32_t>(), ctx->sj_reg_off.as<int64_t>(),
                           ctx->sj_nmax};
        HIPCHK(ctx, ma::launch_map_sj((int)ncols, static_cast<int32_t *>(b_cols), o, cur, old,
                                      ctx->sj_store.as<double>(), ctx->sj_have.as<int32_t>(),
                                      static_cast<double *>(b_x0full), st), "previous start");
    }
    // s_j to keep: the store belongs to the current geometry (re-initialised
    // after the mapping above has read the previous one)
    if (opts.keep_sj && (!ctx->sj_valid || ctx->sj_gen != ctx->generation)) {
        HIPCHK(ctx, hipStreamSynchronize(st), "previous start");
        ctx->sj_valid = false;
        HIPCHK(ctx, ctx->sj_store.reserve(sizeof(double) * (size_t)ctx->M * ctx->nmax), "kept s_j");
        HIPCHK(ctx, ctx->sj_have.reserve(sizeof(int32_t) * (size_t)ctx->M), "kept s_j flags");
        HIPCHK(ctx, ctx->sj_reg_id.reserve(sizeof(int32_t) * ctx->n_atoms), "kept regions");
        HIPCHK(ctx, ctx->sj_reg_off.reserve(sizeof(int64_t) * (ctx->nreg + 1)), "kept regions");
        HIPCHK(ctx, ctx->sj_reg_len.reserve(sizeof(int32_t) * ctx->nreg), "kept regions");
        HIPCHK(ctx, ctx->sj_reg_atoms.reserve(sizeof(int32_t) * ctx->reg_atoms_total), "kept regions");
        HIPCHK(ctx, hipMemsetAsync(ctx->sj_have.p, 0, sizeof(int32_t) * (size_t)ctx->M, st), "kept s_j flags");
        HIPCHK(ctx, hipMemcpyAsync(ctx->sj_reg_id.p, ctx->reg_id.p, sizeof(int32_t) * ctx->n_atoms, hipMemcpyDeviceToDevice, st), "kept regions");
        HIPCHK(ctx, hipMemcpyAsync(ctx->sj_reg_off.p, ctx->reg_off.p, sizeof(int64_t) * (ctx->nreg + 1), hipMemcpyDeviceToDevice, st), "kept regions");
        HIPCHK(ctx, hipMemcpyAsync(ctx->sj_reg_len.p, ctx->reg_len.p, sizeof(int32_t) * ctx->nreg, hipMemcpyDeviceToDevice, st), "kept regions");
        HIPCHK(ctx, hipMemcpyAsync(ctx->sj_reg_atoms.p, ctx->reg_atoms.p, sizeof(int32_t) * ctx->reg_atoms_total, hipMemcpyDeviceToDevice, st), "kept regions");
        ctx->sj_gen = ctx->generation;
        ctx->sj_nmax = ctx->nmax;
        ctx->sj_n_atoms = ctx->n_atoms;
        ctx->sj_o = ctx->o;
        ctx->sj_valid = true;
    }
    // the copies read pageable host vectors: finish them before those go away
    HIPCHK(ctx, hipStreamSynchronize(st), "upload");

    J.cols = static_cast<int32_t *>(b_cols);
    J.order = static_cast<int32_t *>(b_order);
    P.qb_dev = static_cast<int32_t *>(b_qb);
    J.qbounds = P.qb_dev;
    J.c0 = P.ch_c0[0];
    J.cn = P.ch_cn[0];
    J.gstart = static_cast<int32_t *>(b_gstart);
    P.ctl = static_cast<int *>(b_ctl);
    J.queue = P.ctl;
    J.fail = P.ctl + ma::kMaxQueues;
    J.ws = P.kind == ma::kBasisOnchip ? nullptr : static_cast<double *>(b_ws);
    J.mid = static_cast<double *>(b_mid);
    J.eps = eps ? eps : static_cast<double *>(b_eps);
    J.wts = wts ? wts : static_cast<double *>(b_wts);
    J.amp = P.bisect ? b_amp : nullptr;
    J.amp_off = P.bisect ? static_cast<int64_t *>(b_aoff) : nullptr;
    J.stats = col_stats ? col_stats : static_cast<int32_t *>(b_stats);
    P.feat = static_cast<float *>(b_feat);
    P.x0 = static_cast<float *>(b_x0);
    P.lohi = static_cast<double *>(b_lohi);
    P.partial = static_cast<double *>(b_partial);
    P.sums = static_cast<double *>(b_sums);
    J.x0 = learned ? P.x0 : nullptr;
    J.x0full = static_cast<double *>(b_x0full);
    J.sj_store = opts.keep_sj ? ctx->sj_store.as<double>() : nullptr;
    J.sj_have = opts.keep_sj ? ctx->sj_have.as<int32_t>() : nullptr;
    J.sj_near = sj_near;
    J.direct = P.bisect ? 0 : 1;
    J.mu = P.bisect ? 0.0 : mu;
    J.kT = kT;
    J.rho = rho;
    J.pi = pi;
    J.Ecol = static_cast<double *>(b_E);
    J.Ncol = static_cast<double *>(b_N);
    return MA_OK;
}

// The launch sequence of one solve: per chunk the queue reset and the basis
// kernel, then the eigensolver kernel; then the chemical potential, the
// Fermi weighting of the stored amplitudes and the reductions.
hipError_t enqueue_basis(ma_ctx *ctx, const Plan &P, int k)
{
    hipStream_t st = ctx->work_stream();
    const ma::DevJob Jk = P.chunk_job(k);
    hipError_t e = ma::launch_reset(Jk.queue, Jk.fail, k == 0 ? 1 : 0, st);
    if (e != hipSuccess) return e;
    return ma::launch_basis(P.S, Jk, P.kind, (int)std::min<int64_t>(P.slots, P.ch_items[k]), st);
}

hipError_t enqueue_eig(ma_ctx *ctx, const Plan &P, int k, hipStream_t st)
{
    return ma::launch_eig(P.S, P.chunk_job(k), st);
}

hipError_t enqueue_basis0(ma_ctx *ctx, const Plan &P) { return enqueue_basis(ctx, P, 0); }
hipError_t enqueue_eig0(ma_ctx *ctx, const Plan &P) { return enqueue_eig(ctx, P, 0, ctx->work_stream()); }

hipError_t net_refresh_bf16(ma_ctx *ctx, hipStream_t st);

hipError_t enqueue_pre(ma_ctx *ctx, const Plan &P)
{
    hipStream_t st = ctx->work_stream();
    auto &N = ctx->net;
    hipError_t e = ma::launch_features(P.J.cols, P.J.ncols, ctx->o, ctx->geo.as<float>(),
                                       ma::kGeoFeat, N.nf, P.feat, st);
    if (e != hipSuccess) return e;
    if ((e = net_refresh_bf16(ctx, st)) != hipSuccess) return e;
    const float *pr = N.params.as<float>();
    return ma::launch_mlp_infer(P.feat, P.J.ncols, N.nf, N.nf_pad, N.nh, N.no,
                                N.W1t.as<unsigned short>(), pr + N.ob1, N.W2t.as<unsigned short>(),
                                pr + N.ob2, N.W3t.as<unsigned short>(), pr + N.ob3,
                                P.x0, st);
}

hipError_t enqueue_post(ma_ctx *ctx, const Plan &P)
{
    hipStream_t st = ctx->work_stream();
    const ma::DevSystem &S = P.S;
    const ma::DevJob &J = P.J;
    hipError_t e;
    if (P.bisect) {
        if ((e = ma::launch_minmax(J.eps, J.stats, J.ncols, J.nu, P.kT, P.lohi, P.partial, st)) !=
            hipSuccess) return e;
        if ((e = ma::launch_bisect(J.eps, J.wts, J.stats, J.ncols, J.nu, P.kT, P.n_target,
                                   P.lohi, P.partial, st)) != hipSuccess) return e;
        if ((e = ma::launch_rho(S, J, P.lohi, P.kT, P.rho, P.pi, J.Ecol, J.Ncol, st)) != hipSuccess)
            return e;
    }
    return ma::launch_sum2(J.Ecol, J.Ncol, J.ncols, P.sums, st);
}

hipError_t capture(ma_ctx *ctx, const Plan &P, hipError_t (*fn)(ma_ctx *, const Plan &),
                   hipGraphExec_t *exec)
{
    hipStream_t st = ctx->work_stream();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    e = fn(ctx, P);
    hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

template <typename T>
void key_add(std::vector<unsigned char> &k, const T &v)
{
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&v);
    k.insert(k.end(), b, b + sizeof(T));
}

std::vector<unsigned char> graph_key(const ma_ctx *ctx, const Plan &P)
{
    std::vector<unsigned char> k;
    key_add(k, ctx->generation);
    key_add(k, P.J);          // sizes, tolerances, mu, and every device pointer
    key_add(k, P.slots);
    key_add(k, P.kind);
    key_add(k, P.bisect);
    key_add(k, P.kT);
    key_add(k, P.n_target);
    key_add(k, P.rho);
    key_add(k, P.pi);
    return k;
}

// Run the plan; fills the result scalars.  kernel_ms is the basis kernel's
// time and eig_ms the eigensolver kernel's, from HIP events recorded around
// their launches on the stream (summed over chunks).  A single-chunk solve
// with use_graph replays captured graphs; events sit between the graphs.
ma_status run_plan(ma_ctx *ctx, const Plan &P, ma_result *out)
{
    hipStream_t st = ctx->work_stream();
    const bool graphs = P.opts.use_graph && P.nchunks == 1;
    if (graphs) {
        std::vector<unsigned char> key = graph_key(ctx, P);
        if (!ctx->gexec || key != ctx->gkey) {
            ctx->drop_graph();
            hipError_t e = capture(ctx, P, enqueue_basis0, &ctx->gexec);
            if (e == hipSuccess) e = capture(ctx, P, enqueue_eig0, &ctx->gexec1);
            if (e == hipSuccess) e = capture(ctx, P, enqueue_post, &ctx->gexec2);
            if (e == hipSuccess && P.J.x0) e = capture(ctx, P, enqueue_pre, &ctx->gexec0);
            if (e != hipSuccess) {
                ctx->drop_graph();
                return ctx->hip_fail(e, "graph capture");
            }
            ctx->gkey = key;
        }
    }
    float ms = 0.0f;
    double basis_ms = 0.0, eig_ms = 0.0;
    HIPCHK(ctx, hipEventRecord(ctx->ev0, st), "event");
    if (P.J.x0) {
        if (graphs) HIPCHK(ctx, hipGraphLaunch(ctx->gexec0, st), "graph launch");
        else HIPCHK(ctx, enqueue_pre(ctx, P), "start network");
    }
    if (graphs) {
        HIPCHK(ctx, hipEventRecord(ctx->evk0, st), "event");
        HIPCHK(ctx, hipGraphLaunch(ctx->gexec, st), "graph launch");
        HIPCHK(ctx, hipEventRecord(ctx->evk1, st), "event");
        HIPCHK(ctx, hipGraphLaunch(ctx->gexec1, st), "graph launch");
        HIPCHK(ctx, hipEventRecord(ctx->eve1, st), "event");
        HIPCHK(ctx, hipGraphLaunch(ctx->gexec2, st), "graph launch");
    } else {
        // eager: per chunk, events around the basis kernel (stream st) and the
        // eigensolver (st, or the aux stream when pipelined: chunk k's
        // eigensolver runs beside the later basis kernels; chunk k + nbuf
        // reuses chunk k's buffer of the ring only after that eigensolver).
        // The last chunk's eigensolver goes to a second stream, so that it
        // starts when its basis kernel ends instead of queueing behind the
        // previous chunk's: nothing else runs then, and the two eigensolvers
        // write disjoint columns and ring slots.
        if (!P.timed_chunks) {
            // one stream, no per-chunk events (the allocation-free path)
            for (int k = 0; k < P.nchunks; ++k) {
                HIPCHK(ctx, enqueue_basis(ctx, P, k), "basis kernel");
                HIPCHK(ctx, enqueue_eig(ctx, P, k, st), "eigensolver kernel");
            }
        }
        while (P.timed_chunks && (int)ctx->chunk_ev.size() < 6 * P.nchunks) {
            hipEvent_t ev;
            HIPCHK(ctx, hipEventCreate(&ev), "event");
            ctx->chunk_ev.push_back(ev);
        }
        for (int k = 0; P.timed_chunks && k < P.nchunks; ++k) {
            hipEvent_t *ev = &ctx->chunk_ev[6 * k];
            const hipStream_t es = !P.pipelined ? st : (k > 0 && k == P.nchunks - 1) ? ctx->aux2 : ctx->aux;
            if (P.pipelined && k >= P.nbuf)
                HIPCHK(ctx, hipStreamWaitEvent(st, ctx->chunk_ev[6 * (k - P.nbuf) + 5], 0), "wait");
            HIPCHK(ctx, hipEventRecord(ev[0], st), "event");
            HIPCHK(ctx, enqueue_basis(ctx, P, k), "basis kernel");
            HIPCHK(ctx, hipEventRecord(ev[1], st), "event");
            if (P.pipelined) HIPCHK(ctx, hipStreamWaitEvent(es, ev[1], 0), "wait");
            HIPCHK(ctx, hipEventRecord(ev[2], es), "event");
            HIPCHK(ctx, enqueue_eig(ctx, P, k, es), "eigensolver kernel");
            HIPCHK(ctx, hipEventRecord(ev[3], es), "event");
            HIPCHK(ctx, hipEventRecord(ev[5], es), "event");
        }
        if (P.pipelined) {
            HIPCHK(ctx, hipStreamWaitEvent(st, ctx->chunk_ev[6 * (P.nchunks - 1) + 5], 0), "wait");
            if (P.nchunks > 1)
                HIPCHK(ctx, hipStreamWaitEvent(st, ctx->chunk_ev[6 * (P.nchunks - 2) + 5], 0), "wait");
        }
        HIPCHK(ctx, enqueue_post(ctx, P), "launch");
    }
    HIPCHK(ctx, hipEventRecord(ctx->ev1, st), "event");
    double sums[2] = {0, 0}, lohi[2] = {0, 0};
    int ctl[ma::kMaxQueues + 1];
    HIPCHK(ctx, hipMemcpyAsync(sums, P.sums, sizeof sums, hipMemcpyDeviceToHost, st), "copy");
    HIPCHK(ctx, hipMemcpyAsync(ctl, P.ctl, sizeof ctl, hipMemcpyDeviceToHost, st), "copy");
    if (P.bisect) HIPCHK(ctx, hipMemcpyAsync(lohi, P.lohi, sizeof lohi, hipMemcpyDeviceToHost, st), "copy");
    HIPCHK(ctx, hipStreamSynchronize(st), "solve");
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "elapsed");
    out->elapsed_ms = ms;
    if (graphs) {
        HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->evk0, ctx->evk1), "elapsed");
        basis_ms = ms;
        HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->evk1, ctx->eve1), "elapsed");
        eig_ms = ms;
    } else {
        for (int k = 0; P.timed_chunks && k < P.nchunks; ++k) {
            const hipEvent_t *ev = &ctx->chunk_ev[6 * k];
            HIPCHK(ctx, hipEventElapsedTime(&ms, ev[0], ev[1]), "elapsed");
            basis_ms += ms;
            HIPCHK(ctx, hipEventElapsedTime(&ms, ev[2], ev[3]), "elapsed");
            eig_ms += ms;
        }
    }
    out->kernel_ms = basis_ms;
    out->eig_ms = eig_ms;
    out->energy = P.opts.spin * sums[0];
    out->n_elec = P.opts.spin * sums[1];
    out->mu = P.bisect ? 0.5 * (lohi[0] + lohi[1]) : P.mu;
    const int failc = ctl[ma::kMaxQueues];
    if (failc != INT_MAX) {
        int32_t st4[4] = {0, 0, 0, 0};
        HIPCHK(ctx, hipMemcpy(st4, P.J.stats + (int64_t)failc * ma::kStats, sizeof st4, hipMemcpyDeviceToHost), "copy");
        const ma_status s = st4[3] == -4 ? MA_ENOTPD : MA_ENOCONV;
        return ctx->fail(s, "column %d (output row %d): %s after %d CG iterations", P.hcols[failc],
                         failc, s == MA_ENOTPD ? "S_A or the reduced overlap not positive definite"
                                               : "CG did not converge",
                         st4[1]);
    }
    return MA_OK;
}

}  // namespace

extern "C" {

MA_API ma_status ma_solve_columns(ma_ctx *ctx, int64_t ncols, const int32_t *cols, int32_t p,
                                  int32_t q, double mu, double kT, const ma_opts *opts_in,
                                  ma_result *out)
{
    if (!ctx) return MA_EINVAL;
    if (!out) return ctx->fail(MA_EINVAL, "null result");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ctx->last_valid = ctx->last_ritz = false;
    Plan P;
    BufSource src;
    if (ctx->user_ws) {
        src.base = ctx->user_ws;
        src.cap = ctx->user_ws_bytes;
    }
    ma_status s = make_plan(ctx, ncols, cols, p, q, mu, kT, opts_in, out->rho, out->pi, out->eps,
                            out->wts, out->col_stats, out->sj_near, 0, -1, P, &src);
    if (s != MA_OK) return s;
    s = run_plan(ctx, P, out);
    if (s == MA_OK) {
        ctx->last_ritz = true;
        ctx->lastS = P.S;
        ctx->lastJ = P.J;
    }
    if (s == MA_OK && P.bisect) {
        ctx->last_valid = true;
        ctx->lastS = P.S;
        ctx->lastJ = P.J;
        ctx->last_lohi = P.lohi;
        ctx->last_partial = P.partial;
        ctx->last_sums = P.sums;
    }
    return s;
}

MA_API ma_status ma_find_mu(ma_ctx *ctx, double n_target, double kT, double spin,
                            ma_result *out)
{
    if (!ctx) return MA_EINVAL;
    if (!out) return ctx->fail(MA_EINVAL, "null result");
    if (!ctx->last_valid)
        return ctx->fail(MA_ESTATE, "no bisected solve to reuse (the last solve was given mu, "
                         "failed, or was followed by a build or workspace change)");
    if (!(kT > 0) || !std::isfinite(kT)) return ctx->fail(MA_EINVAL, "kT must be positive");
    if (!std::isfinite(n_target)) return ctx->fail(MA_EINVAL, "n_target must be finite");
    if (!std::isfinite(spin)) return ctx->fail(MA_EINVAL, "spin must be finite");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const ma::DevSystem &S = ctx->lastS;
    const ma::DevJob &J = ctx->lastJ;
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    HIPCHK(ctx, hipEventRecord(ctx->ev0, st), "event");
    HIPCHK(ctx, ma::launch_minmax(J.eps, J.stats, J.ncols, J.nu, kT, ctx->last_lohi,
                                  ctx->last_partial, st), "bracket");
    HIPCHK(ctx, ma::launch_bisect(J.eps, J.wts, J.stats, J.ncols, J.nu, kT, n_target,
                                  ctx->last_lohi, ctx->last_partial, st), "bisection");
    HIPCHK(ctx, ma::launch_rho(S, J, ctx->last_lohi, kT, out->rho, out->pi, J.Ecol, J.Ncol, st),
           "rho");
    HIPCHK(ctx, ma::launch_sum2(J.Ecol, J.Ncol, J.ncols, ctx->last_sums, st), "sums");
    HIPCHK(ctx, hipEventRecord(ctx->ev1, st), "event");
    double sums[2] = {0, 0}, lohi[2] = {0, 0};
    HIPCHK(ctx, hipMemcpyAsync(sums, ctx->last_sums, sizeof sums, hipMemcpyDeviceToHost, st), "copy");
    HIPCHK(ctx, hipMemcpyAsync(lohi, ctx->last_lohi, sizeof lohi, hipMemcpyDeviceToHost, st), "copy");
    HIPCHK(ctx, hipStreamSynchronize(st), "find_mu");
    float ms = 0.0f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "elapsed");
    out->elapsed_ms = ms;
    out->kernel_ms = 0.0;
    out->eig_ms = 0.0;
    out->energy = spin * sums[0];
    out->n_elec = spin * sums[1];
    out->mu = 0.5 * (lohi[0] + lohi[1]);
    return MA_OK;
}

MA_API ma_status ma_forces(ma_ctx *ctx, const double *dH, const double *dS, const double *rho,
                           const double *pi, double spin, double *forces)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->built) return ctx->fail(MA_ESTATE, "ma_build_system has not succeeded");
    if (!dH || !dS || !rho || !pi || !forces) return ctx->fail(MA_EINVAL, "null array");
    if (!std::isfinite(spin)) return ctx->fail(MA_EINVAL, "spin must be finite");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    HIPCHK(ctx, ma::launch_forces(ctx->n_atoms, ctx->o, ctx->blk_ptr.as<int64_t>(),
                                  ctx->blk_col.as<int32_t>(), ctx->blk_t.as<int32_t>(), dH, dS, rho,
                                  pi, spin, forces, st), "forces");
    HIPCHK(ctx, hipStreamSynchronize(st), "forces");
    return MA_OK;
}

MA_API ma_status ma_dos(ma_ctx *ctx, int64_t n_energies, const double *energies, double eta,
                        double spin, double *dos)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->last_ritz) return ctx->fail(MA_ESTATE, "no solve whose Ritz data are kept");
    if (n_energies < 1 || n_energies > INT_MAX || !energies || !dos)
        return ctx->fail(MA_EINVAL, "need n_energies >= 1 and host arrays");
    if (!(eta > 0) || !std::isfinite(eta) || !std::isfinite(spin))
        return ctx->fail(MA_EINVAL, "eta must be positive");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const ma::DevJob &J = ctx->lastJ;
    const int nE = (int)n_energies;
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    HIPCHK(ctx, ctx->dos_E.reserve(sizeof(double) * nE), "energies");
    HIPCHK(ctx, ctx->dos_out.reserve(sizeof(double) * nE), "dos");
    HIPCHK(ctx, ctx->dos_part.reserve(sizeof(double) * std::max<size_t>(1, ma::dos_partial_doubles(J.ncols, J.nu, nE))), "dos partials");
    HIPCHK(ctx, hipMemcpyAsync(ctx->dos_E.p, energies, sizeof(double) * nE, hipMemcpyHostToDevice, st), "energies");
    HIPCHK(ctx, ma::launch_dos(J.eps, J.wts, J.stats, J.ncols, J.nu, ctx->dos_E.as<double>(), nE, eta,
                               spin, ctx->dos_part.as<double>(), ctx->dos_out.as<double>(), st), "dos");
    HIPCHK(ctx, hipMemcpyAsync(dos, ctx->dos_out.p, sizeof(double) * nE, hipMemcpyDeviceToHost, st), "dos");
    HIPCHK(ctx, hipStreamSynchronize(st), "dos");
    return MA_OK;
}

MA_API ma_status ma_green(ma_ctx *ctx, double z_re, double z_im, double *g_re, double *g_im)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->last_valid)
        return ctx->fail(MA_ESTATE, "no bisected solve whose amplitudes are kept");
    if (!std::isfinite(z_re) || !std::isfinite(z_im) || z_im == 0.0)
        return ctx->fail(MA_EINVAL, "z must be finite with a nonzero imaginary part");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    HIPCHK(ctx, ma::launch_green(ctx->lastS, ctx->lastJ, z_re, z_im, g_re, g_im, st), "green");
    HIPCHK(ctx, hipStreamSynchronize(st), "green");
    return MA_OK;
}

MA_API size_t ma_workspace_size(ma_ctx *ctx, int64_t ncols, const int32_t *cols, int32_t p,
                                int32_t q, double mu, const ma_opts *opts)
{
    if (!ctx) return 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return 0;
    Plan P;
    BufSource src;
    src.size_only = true;
    src.cap = SIZE_MAX;
    if (make_plan(ctx, ncols, cols, p, q, mu, 1.0, opts, nullptr, nullptr, nullptr, nullptr,
                  nullptr, nullptr, 0, -1, P, &src) != MA_OK)
        return 0;
    return P.bytes;
}

MA_API ma_status ma_set_workspace(ma_ctx *ctx, void *device_ptr, size_t bytes)
{
    if (!ctx) return MA_EINVAL;
    if ((device_ptr == nullptr) != (bytes == 0))
        return ctx->fail(MA_EINVAL, "a workspace needs both a pointer and a size");
    if (reinterpret_cast<uintptr_t>(device_ptr) % 256 != 0)
        return ctx->fail(MA_EINVAL, "the workspace must be 256-byte aligned");
    ctx->last_valid = ctx->last_ritz = false;
    ctx->drop_graph();
    ctx->user_ws = static_cast<char *>(device_ptr);
    ctx->user_ws_bytes = bytes;
    return MA_OK;
}

MA_API ma_status ma_solve_columns_noalloc(ma_ctx *ctx, int64_t ncols, const int32_t *cols,
                                          int32_t p, int32_t q, double mu, double kT,
                                          const ma_opts *opts_in, ma_result *out)
{
    if (!ctx) return MA_EINVAL;
    if (!out) return ctx->fail(MA_EINVAL, "null result");
    if (!ctx->scratch) return ctx->fail(MA_ESTATE, "no scratch on this device");
    ma_opts o;
    ma_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.start != MA_START_ZERO)
        return ctx->fail(MA_EINVAL, "the allocation-free solve supports the zero CG start only");
    if (out->sj_near) return ctx->fail(MA_EINVAL, "the allocation-free solve does not write sj_near");
    if (o.keep_sj) return ctx->fail(MA_EINVAL, "the allocation-free solve does not keep s_j");
    o.use_graph = 0;   // instantiating a graph allocates
    o.pipeline = 0;    // one stream, chunks in sequence over one chunk buffer
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ctx->last_valid = ctx->last_ritz = false;
    Plan P;
    BufSource src;
    src.base = static_cast<char *>(ctx->scratch);
    src.cap = ctx->scratch_bytes;
    src.limited = true;
    ma_status s = make_plan(ctx, ncols, cols, p, q, mu, kT, &o, out->rho, out->pi, out->eps,
                            out->wts, out->col_stats, nullptr, 0, -1, P, &src);
    if (s != MA_OK) return s;
    P.timed_chunks = false;
    s = run_plan(ctx, P, out);
    out->kernel_ms = 0.0;
    out->eig_ms = 0.0;
    return s;
}

MA_API ma_status ma_set_tuning(ma_ctx *ctx, int32_t p, int32_t q, int32_t precision,
                               int32_t slots_per_cu, int32_t schedule, int32_t basis_kernel,
                               int32_t pipeline)
{
    if (!ctx) return MA_EINVAL;
    if (slots_per_cu < 1 || schedule < 0 || schedule > MA_SCHED_SPATIAL ||
        basis_kernel < MA_BASIS_AUTO || basis_kernel > MA_BASIS_ATOM || pipeline < -1)
        return ctx->fail(MA_EINVAL, "invalid tuning");
    for (auto &t : ctx->tunes)
        if (t.p == p && t.q == q && t.prec == precision) {
            t.slots = slots_per_cu;
            t.sched = schedule;
            t.kernel = basis_kernel;
            t.pipe = pipeline;
            return MA_OK;
        }
    ctx->tunes.push_back({p, q, precision, slots_per_cu, schedule, basis_kernel, pipeline});
    return MA_OK;
}

MA_API ma_status ma_autotune(ma_ctx *ctx, int64_t ncols, const int32_t *cols, int32_t p, int32_t q,
                             double mu, double kT, const ma_opts *opts_in, int32_t reps,
                             ma_tuning *out)
{
    if (!ctx) return MA_EINVAL;
    if (!out || reps < 1) return ctx->fail(MA_EINVAL, "null result or reps < 1");
    if (!std::isfinite(mu)) return ctx->fail(MA_EINVAL, "autotuning needs a finite mu");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ctx->last_valid = ctx->last_ritz = false;
    BufSource src;
    if (ctx->user_ws) {
        src.base = ctx->user_ws;
        src.cap = ctx->user_ws_bytes;
    }
    ma_opts o;
    ma_default_opts(&o);
    if (opts_in) o = *opts_in;
    o.keep_sj = 0;   // timing solves leave the kept s_j alone
    o.use_graph = 0;
    const int pipe_on = o.pipeline >= 0 ? o.pipeline : 4;
    std::memset(out, 0, sizeof(*out));
    out->best_ms = INFINITY;
    // one timed candidate: best of reps over the whole solve (with
    // pipelining, a basis kernel that leaves no room for the eigensolver
    // beside it can be faster alone and slower in the solve)
    auto trial = [&](int kern, int sched, int bpc, int pipe, double &best) -> ma_status {
        o.basis_kernel = kern;
        o.pipeline = pipe;
        Plan P;
        BufSource run = src;
        ma_status s = make_plan(ctx, ncols, cols, p, q, mu, kT, &o, nullptr, nullptr, nullptr,
                                nullptr, nullptr, nullptr, bpc, sched, P, &run);
        if (s != MA_OK) return s;
        best = INFINITY;
        for (int r = 0; r < reps; ++r) {
            ma_result res{};
            s = run_plan(ctx, P, &res);
            if (s != MA_OK) return s;
            best = std::min(best, res.elapsed_ms);
        }
        if (out->n_tried < 64) {
            const int t = out->n_tried++;
            out->tried_slots[t] = bpc;
            out->tried_schedule[t] = sched;
            out->tried_kernel[t] = kern;
            out->tried_pipeline[t] = pipe;
            out->tried_ms[t] = best;
        }
        if (best < out->best_ms) {
            out->best_ms = best;
            out->slots_per_cu = bpc;
            out->schedule = sched;
            out->basis_kernel = kern;
            out->pipeline = pipe;
        }
        return MA_OK;
    };
    for (int kern = MA_BASIS_ONCHIP; kern <= MA_BASIS_ATOM; ++kern) {
        if (kern == MA_BASIS_ONCHIP && !ma::basis_small_fits(ctx->nmax, p + q, q, ctx->o)) continue;
        if (kern == MA_BASIS_GROUP && !ma::basis_group_fits(ctx->nmax, p + q, ctx->o)) continue;
        if (kern == MA_BASIS_ATOM && !ma::basis_atom_fits(ctx->nmax, p + q, ctx->o, o.precision)) continue;
        o.basis_kernel = kern;
        o.pipeline = pipe_on;
        // occupancy limit of this kernel and shape
        Plan P0;
        BufSource sz;
        sz.size_only = true;
        sz.cap = SIZE_MAX;
        ma_status s = make_plan(ctx, ncols, cols, p, q, mu, kT, &o, nullptr, nullptr, nullptr,
                                nullptr, nullptr, nullptr, 1 << 20, MA_SCHED_LPT, P0, &sz);
        if (s != MA_OK) return s;
        const int max_bpc = std::max(1, P0.slots / std::max(1, ctx->cu_count));
        double kbest = INFINITY;
        int kb_sched = 0, kb_bpc = 1;
        for (int sched = 0; sched <= MA_SCHED_SPATIAL; ++sched)
            for (int bpc = 1; bpc <= max_bpc && out->n_tried < 63; ++bpc) {
                double best;
                s = trial(kern, sched, bpc, pipe_on, best);
                if (s != MA_OK) return s;
                if (best < kbest) {
                    kbest = best;
                    kb_sched = sched;
                    kb_bpc = bpc;
                }
            }
        // the kernel's fastest workgroup count with the chunks in sequence,
        // every schedule
        for (int sched = 0; pipe_on >= 2 && std::isfinite(kbest) && sched <= MA_SCHED_SPATIAL &&
                            out->n_tried < 64; ++sched) {
            double best;
            s = trial(kern, sched, kb_bpc, 0, best);
            if (s != MA_OK) return s;
        }
        (void)kb_sched;
    }
    // The schedules differ in how the columns in flight share the caches,
    // which a trial on a sample of the columns measures only roughly (on the
    // 262,144-atom cell LPT order is 6 % slower than Morton order, but on a
    // sample the two can come out within 1 %).  When the trials ran on a
    // sample, among those with the best one's kernel, workgroups per CU and
    // pipelining that lie within 2 % of it, the schedule is taken in the order
    // spatial, input, per-XCD input, per-XCD LPT, LPT.  Trials on every
    // column measure the solve itself and decide alone.
    if (cols && ncols < ctx->M) {
        static const int pref[5] = {4, 1, 2, 3, 0};   // rank of MA_SCHED_LPT .. MA_SCHED_SPATIAL
        int bi = -1;
        for (int t = 0; t < out->n_tried; ++t)
            if (out->tried_kernel[t] == out->basis_kernel && out->tried_slots[t] == out->slots_per_cu &&
                out->tried_pipeline[t] == out->pipeline && out->tried_schedule[t] == out->schedule)
                bi = t;
        const double lim = bi >= 0 ? 1.02 * out->tried_ms[bi] : 0.0;
        for (int t = 0; bi >= 0 && t < out->n_tried; ++t)
            if (out->tried_kernel[t] == out->basis_kernel && out->tried_slots[t] == out->slots_per_cu &&
                out->tried_pipeline[t] == out->pipeline && out->tried_ms[t] <= lim &&
                pref[out->tried_schedule[t]] < pref[out->schedule]) {
                out->schedule = out->tried_schedule[t];
                out->best_ms = out->tried_ms[t];
            }
    }
    return ma_set_tuning(ctx, p, q, o.precision, out->slots_per_cu, out->schedule,
                         out->basis_kernel, out->pipeline);
}

}  // extern "C"

namespace {

ma_status net_shape(ma_ctx *ctx)
{
    auto &N = ctx->net;
    N.nf = ma::kGeoFeat + ctx->o;
    N.nh = ma::kHidden;
    N.no = ma::kNbOut * ctx->o;
    N.nf_pad = (N.nf + 15) / 16 * 16;
    N.no_pad = (N.no + 15) / 16 * 16;
    N.oW1 = 0;
    N.ob1 = N.oW1 + (int64_t)N.nf * N.nh;
    N.oW2 = N.ob1 + N.nh;
    N.ob2 = N.oW2 + (int64_t)N.nh * N.nh;
    N.oW3 = N.ob2 + N.nh;
    N.ob3 = N.oW3 + (int64_t)N.nh * N.no;
    N.P = N.ob3 + N.no;
    HIPCHK(ctx, N.params.reserve(sizeof(float) * N.P), "network");
    HIPCHK(ctx, N.grad.reserve(sizeof(float) * N.P), "network");
    HIPCHK(ctx, N.m.reserve(sizeof(float) * N.P), "network");
    HIPCHK(ctx, N.v.reserve(sizeof(float) * N.P), "network");
    HIPCHK(ctx, N.W1t.reserve(sizeof(unsigned short) * (size_t)N.nh * N.nf_pad), "network");
    HIPCHK(ctx, N.W2t.reserve(sizeof(unsigned short) * (size_t)N.nh * N.nh), "network");
    HIPCHK(ctx, N.W3t.reserve(sizeof(unsigned short) * (size_t)N.no_pad * N.nh), "network");
    return MA_OK;
}

hipError_t net_refresh_bf16(ma_ctx *ctx, hipStream_t st)
{
    auto &N = ctx->net;
    const float *p = N.params.as<float>();
    hipError_t e = ma::launch_to_bf16_t(p + N.oW1, N.nf, N.nh, N.nf_pad, N.nh, N.W1t.as<unsigned short>(), st);
    if (e == hipSuccess) e = ma::launch_to_bf16_t(p + N.oW2, N.nh, N.nh, N.nh, N.nh, N.W2t.as<unsigned short>(), st);
    if (e == hipSuccess) e = ma::launch_to_bf16_t(p + N.oW3, N.nh, N.no, N.nh, N.no_pad, N.W3t.as<unsigned short>(), st);
    return e;
}

ma_status net_workspace(ma_ctx *ctx, int64_t n)
{
    auto &N = ctx->net;
    HIPCHK(ctx, N.Xb.reserve(sizeof(float) * (size_t)n * N.nf), "training workspace");
    HIPCHK(ctx, N.Tb.reserve(sizeof(float) * (size_t)n * N.no), "training workspace");
    HIPCHK(ctx, N.Z1.reserve(sizeof(float) * (size_t)n * N.nh), "training workspace");
    HIPCHK(ctx, N.A1.reserve(sizeof(float) * (size_t)n * N.nh), "training workspace");
    HIPCHK(ctx, N.Z2.reserve(sizeof(float) * (size_t)n * N.nh), "training workspace");
    HIPCHK(ctx, N.A2.reserve(sizeof(float) * (size_t)n * N.nh), "training workspace");
    HIPCHK(ctx, N.Yb.reserve(sizeof(float) * (size_t)n * N.no), "training workspace");
    HIPCHK(ctx, N.dY.reserve(sizeof(float) * (size_t)n * N.no), "training workspace");
    HIPCHK(ctx, N.dA.reserve(sizeof(float) * (size_t)n * N.nh), "training workspace");
    HIPCHK(ctx, N.partial.reserve(sizeof(double) * 256), "training workspace");
    return MA_OK;
}

// FP32 forward for n rows of x into y (activations kept for the backward pass).
hipError_t net_forward_f32(ma_ctx *ctx, const float *x, int64_t n, float *y, hipStream_t st)
{
    auto &N = ctx->net;
    const float *p = N.params.as<float>();
    hipError_t e = ma::launch_gemm((int)n, N.nh, N.nf, x, N.nf, 1, nullptr, p + N.oW1, N.nh, 1,
                                   p + N.ob1, 0.f, N.A1.as<float>(), N.nh, N.Z1.as<float>(), st);
    if (e == hipSuccess)
        e = ma::launch_gemm((int)n, N.nh, N.nh, N.A1.as<float>(), N.nh, 1, nullptr, p + N.oW2, N.nh, 1,
                            p + N.ob2, 0.f, N.A2.as<float>(), N.nh, N.Z2.as<float>(), st);
    if (e == hipSuccess)
        e = ma::launch_gemm((int)n, N.no, N.nh, N.A2.as<float>(), N.nh, 1, nullptr, p + N.oW3, N.no, 1,
                            p + N.ob3, 0.f, y, N.no, nullptr, st);
    return e;
}

// Loss and gradient of the mean squared error on n rows; optional Adam step.
ma_status net_train_core(ma_ctx *ctx, const float *x, const float *t, const int32_t *idx, int64_t n,
                         int64_t n_rows, bool update, float lr, double *loss, float *grad_host)
{
    auto &N = ctx->net;
    if (!N.ready) return ctx->fail(MA_ESTATE, "no start network (ma_mlp_init or ma_mlp_set_params)");
    if (!x || !t || n < 1 || n > INT_MAX) return ctx->fail(MA_EINVAL, "invalid training batch");
    if (n_rows < 1 || (!idx && n > n_rows))
        return ctx->fail(MA_EINVAL, "batch of %lld rows from a table of %lld", (long long)n,
                         (long long)n_rows);
    ma_status s = net_workspace(ctx, n);
    if (s != MA_OK) return s;
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    const float *X = x, *T = t;
    if (idx) {
        // the device indices are checked by the gather: one outside the
        // table fails the call before any update
        HIPCHK(ctx, N.bad.reserve(sizeof(int)), "index flag");
        HIPCHK(ctx, hipMemsetAsync(N.bad.p, 0, sizeof(int), st), "index flag");
        HIPCHK(ctx, ma::launch_gather_rows(x, idx, n, N.nf, n_rows, N.Xb.as<float>(),
                                           N.bad.as<int>(), st), "gather");
        HIPCHK(ctx, ma::launch_gather_rows(t, idx, n, N.no, n_rows, N.Tb.as<float>(),
                                           N.bad.as<int>(), st), "gather");
        int bad = 0;
        HIPCHK(ctx, hipMemcpyAsync(&bad, N.bad.p, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
        HIPCHK(ctx, hipStreamSynchronize(st), "gather");
        if (bad) return ctx->fail(MA_EINVAL, "a row index is outside the table of %lld rows",
                                  (long long)n_rows);
        X = N.Xb.as<float>();
        T = N.Tb.as<float>();
    }
    float *p = N.params.as<float>(), *g = N.grad.as<float>();
    const int nn = (int)n;
    HIPCHK(ctx, net_forward_f32(ctx, X, n, N.Yb.as<float>(), st), "forward");
    HIPCHK(ctx, ma::launch_mse(N.Yb.as<float>(), T, nullptr, n, N.no, N.dY.as<float>(),
                               N.partial.as<double>(), 256, st), "loss");
    // layer 3
    HIPCHK(ctx, ma::launch_gemm(N.nh, N.no, nn, N.A2.as<float>(), 1, N.nh, nullptr, N.dY.as<float>(),
                                N.no, 1, nullptr, 0.f, g + N.oW3, N.no, nullptr, st), "backward");
    HIPCHK(ctx, ma::launch_colsum(N.dY.as<float>(), n, N.no, g + N.ob3, st), "backward");
    HIPCHK(ctx, ma::launch_gemm(nn, N.nh, N.no, N.dY.as<float>(), N.no, 1, nullptr, p + N.oW3, 1, N.no,
                                nullptr, 0.f, N.dA.as<float>(), N.nh, nullptr, st), "backward");
    // layer 2
    HIPCHK(ctx, ma::launch_silu_bwd(N.dA.as<float>(), N.Z2.as<float>(), n * N.nh, st), "backward");
    HIPCHK(ctx, ma::launch_gemm(N.nh, N.nh, nn, N.A1.as<float>(), 1, N.nh, nullptr, N.dA.as<float>(),
                                N.nh, 1, nullptr, 0.f, g + N.oW2, N.nh, nullptr, st), "backward");
    HIPCHK(ctx, ma::launch_colsum(N.dA.as<float>(), n, N.nh, g + N.ob2, st), "backward");
    float *dA1 = N.Z2.as<float>();   // Z2 is no longer needed
    HIPCHK(ctx, ma::launch_gemm(nn, N.nh, N.nh, N.dA.as<float>(), N.nh, 1, nullptr, p + N.oW2, 1, N.nh,
                                nullptr, 0.f, dA1, N.nh, nullptr, st), "backward");
    // layer 1
    HIPCHK(ctx, ma::launch_silu_bwd(dA1, N.Z1.as<float>(), n * N.nh, st), "backward");
    HIPCHK(ctx, ma::launch_gemm(N.nf, N.nh, nn, X, 1, N.nf, nullptr, dA1, N.nh, 1, nullptr, 0.f,
                                g + N.oW1, N.nh, nullptr, st), "backward");
    HIPCHK(ctx, ma::launch_colsum(dA1, n, N.nh, g + N.ob1, st), "backward");
    if (update) {
        N.step += 1;
        HIPCHK(ctx, ma::launch_adam(p, g, N.m.as<float>(), N.v.as<float>(), N.P, lr, 0.9f, 0.999f,
                                    1e-8f, N.step, st), "adam");
        N.bf16_dirty = true;
    }
    double part[256];
    HIPCHK(ctx, hipMemcpyAsync(part, N.partial.p, sizeof part, hipMemcpyDeviceToHost, st), "copy");
    if (grad_host)
        HIPCHK(ctx, hipMemcpyAsync(grad_host, g, sizeof(float) * N.P, hipMemcpyDeviceToHost, st), "copy");
    HIPCHK(ctx, hipStreamSynchronize(st), "training step");
    if (loss) {
        double sum = 0.0;
        for (int b = 0; b < 256; ++b) sum += part[b];
        *loss = sum / ((double)n * N.no);
    }
    return MA_OK;
}

}  // namespace

extern "C" {

MA_API ma_status ma_mlp_shape_of(const ma_ctx *ctx, ma_mlp_shape *out)
{
    if (!ctx || !out) return MA_EINVAL;
    if (!ctx->built) return MA_ESTATE;
    out->n_in = ma::kGeoFeat + ctx->o;
    out->n_hidden = ma::kHidden;
    out->n_out = ma::kNbOut * ctx->o;
    out->n_params = (int64_t)out->n_in * out->n_hidden + out->n_hidden +
                    (int64_t)out->n_hidden * out->n_hidden + out->n_hidden +
                    (int64_t)out->n_hidden * out->n_out + out->n_out;
    return MA_OK;
}

MA_API ma_status ma_mlp_init(ma_ctx *ctx, uint64_t seed)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->built) return ctx->fail(MA_ESTATE, "build a system first (the network's shape follows o)");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ma_status s = net_shape(ctx);
    if (s != MA_OK) return s;
    auto &N = ctx->net;
    std::vector<float> h(N.P, 0.0f);
    // splitmix64 stream -> Box-Muller normals
    uint64_t state = seed;
    auto next = [&]() {
        uint64_t z = (state += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int64_t off, int64_t count, double sd) {
        for (int64_t i = 0; i < count; ++i) {
            const double u1 = next(), u2 = next();
            h[off + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2));
        }
    };
    fill(N.oW1, (int64_t)N.nf * N.nh, std::sqrt(2.0 / N.nf));
    fill(N.oW2, (int64_t)N.nh * N.nh, std::sqrt(2.0 / N.nh));
    fill(N.oW3, (int64_t)N.nh * N.no, std::sqrt(1.0 / N.nh));
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, hipMemcpyAsync(N.params.p, h.data(), sizeof(float) * N.P, hipMemcpyHostToDevice, st), "upload");
    std::vector<float> z(N.P, 0.0f);
    HIPCHK(ctx, hipMemcpyAsync(N.m.p, z.data(), sizeof(float) * N.P, hipMemcpyHostToDevice, st), "upload");
    HIPCHK(ctx, hipMemcpyAsync(N.v.p, z.data(), sizeof(float) * N.P, hipMemcpyHostToDevice, st), "upload");
    HIPCHK(ctx, hipStreamSynchronize(st), "upload");
    N.step = 0;
    N.ready = true;
    N.bf16_dirty = true;
    ctx->drop_graph();
    return MA_OK;
}

MA_API ma_status ma_mlp_set_params(ma_ctx *ctx, const float *params, int64_t count)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->built) return ctx->fail(MA_ESTATE, "build a system first");
    ma_status s = net_shape(ctx);
    if (s != MA_OK) return s;
    auto &N = ctx->net;
    if (!params || count != N.P) return ctx->fail(MA_EINVAL, "expected %lld parameters", (long long)N.P);
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) return ctx->fail(MA_EINVAL, "non-finite parameter %lld", (long long)i);
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, hipMemcpyAsync(N.params.p, params, sizeof(float) * N.P, hipMemcpyHostToDevice, st), "upload");
    std::vector<float> z(N.P, 0.0f);
    HIPCHK(ctx, hipMemcpyAsync(N.m.p, z.data(), sizeof(float) * N.P, hipMemcpyHostToDevice, st), "upload");
    HIPCHK(ctx, hipMemcpyAsync(N.v.p, z.data(), sizeof(float) * N.P, hipMemcpyHostToDevice, st), "upload");
    HIPCHK(ctx, hipStreamSynchronize(st), "upload");
    N.step = 0;
    N.ready = true;
    N.bf16_dirty = true;
    return MA_OK;
}

MA_API ma_status ma_mlp_get_params(const ma_ctx *ctx, float *params, int64_t count)
{
    if (!ctx) return MA_EINVAL;
    const auto &N = ctx->net;
    if (!N.ready) return MA_ESTATE;
    if (!params || count != N.P) return MA_EINVAL;
    if (hipMemcpy(params, N.params.p, sizeof(float) * N.P, hipMemcpyDeviceToHost) != hipSuccess)
        return MA_EDEVICE;
    return MA_OK;
}

MA_API ma_status ma_column_features(ma_ctx *ctx, int64_t ncols, const int32_t *cols, float *feat)
{
    if (!ctx) return MA_EINVAL;
    if (!ctx->built || !ctx->have_geo) return ctx->fail(MA_ESTATE, "no system with positions");
    if (!cols || !feat || ncols < 1 || ncols > INT_MAX) return ctx->fail(MA_EINVAL, "invalid arguments");
    for (int64_t c = 0; c < ncols; ++c)
        if (cols[c] < 0 || cols[c] >= ctx->M) return ctx->fail(MA_EINVAL, "column out of range");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    HIPCHK(ctx, ctx->cols.reserve(sizeof(int32_t) * ncols), "cols");
    HIPCHK(ctx, hipMemcpyAsync(ctx->cols.p, cols, sizeof(int32_t) * ncols, hipMemcpyHostToDevice, st), "cols");
    HIPCHK(ctx, ma::launch_features(ctx->cols.as<int32_t>(), (int)ncols, ctx->o, ctx->geo.as<float>(),
                                    ma::kGeoFeat, ma::kGeoFeat + ctx->o, feat, st), "descriptors");
    HIPCHK(ctx, hipStreamSynchronize(st), "descriptors");
    ctx->drop_graph();   // the column buffer of a captured solve was rewritten
    return MA_OK;
}

MA_API ma_status ma_mlp_forward(ma_ctx *ctx, const float *x, int64_t n, float *y, int32_t bf16)
{
    if (!ctx) return MA_EINVAL;
    auto &N = ctx->net;
    if (!N.ready) return ctx->fail(MA_ESTATE, "no start network");
    if (!x || !y || n < 1 || n > INT_MAX) return ctx->fail(MA_EINVAL, "invalid arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = ctx->work_stream();
    HIPCHK(ctx, ctx->after_caller(), "stream order");
    if (bf16) {
        HIPCHK(ctx, net_refresh_bf16(ctx, st), "bf16 weights");
        const float *p = N.params.as<float>();
        HIPCHK(ctx, ma::launch_mlp_infer(x, n, N.nf, N.nf_pad, N.nh, N.no, N.W1t.as<unsigned short>(),
                                         p + N.ob1, N.W2t.as<unsigned short>(), p + N.ob2,
                                         N.W3t.as<unsigned short>(), p + N.ob3, y, st), "inference");
    } else {
        ma_status s = net_workspace(ctx, n);
        if (s != MA_OK) return s;
        HIPCHK(ctx, net_forward_f32(ctx, x, n, y, st), "forward");
    }
    HIPCHK(ctx, hipStreamSynchronize(st), "forward");
    return MA_OK;
}

MA_API ma_status ma_mlp_loss_grad(ma_ctx *ctx, const float *x, const float *t, int64_t n_rows,
                                  const int32_t *idx, int64_t n, double *loss, float *grad)
{
    if (!ctx) return MA_EINVAL;
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return net_train_core(ctx, x, t, idx, n, n_rows, false, 0.0f, loss, grad);
}

MA_API ma_status ma_mlp_train_step(ma_ctx *ctx, const float *x, const float *t, int64_t n_rows,
                                   const int32_t *idx, int64_t n, float lr, double *loss)
{
    if (!ctx) return MA_EINVAL;
    if (!(lr > 0)) return ctx->fail(MA_EINVAL, "lr must be positive");
    HIPCHK(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return net_train_core(ctx, x, t, idx, n, n_rows, true, lr, loss, nullptr);
}

}  // extern "C"
