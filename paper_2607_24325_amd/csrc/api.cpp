// Host runtime of libhweno: the C ABI of include/hweno.h.  Owns the device
// buffers of a handle, the per-problem table, the tile and reduction work
// lists, and the HIP graph of one SSP-RK3 step; every compute step runs in
// the HIP kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hweno.h"
#include "internal.h"

using namespace hweno;

struct hweno_handle {
    hweno_config cfg{};
    std::vector<hweno_problem> probs;
    int nprob = 0, dim = 1, flux = 0, K = 1, D = 1, nvar = 2, prec = 0;
    size_t su = 8, sd = 8;  // bytes per stored average / derivative value
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* ws = nullptr;
    bool own_ws = false;
    size_t ws_bytes = 0;
    StateBuf U[3]{};
    void* H = nullptr;
    ProbDev* d_probs = nullptr;
    StepCtl* d_ctl = nullptr;
    std::vector<ProbDev> h_probs;   // static fields (offsets, sizes, spacing)
    std::vector<int64_t> ncell;
    // work lists
    void* d_tiles = nullptr;        // step list followed by the per-problem list
    size_t tiles_cap = 0;           // capacity in tiles
    int ntiles_step = 0;
    std::vector<int> tile_begin, tile_count;  // per problem, in the per-problem list
    Chunk* d_chunks = nullptr;
    int nchunks = 0;
    double* d_stage = nullptr;      // staging for set/get_state and rhs (double)
    size_t stage_elems = 0;
    std::vector<char> state_set;
    // Step graphs: the full step, and the step without the reduction of
    // stale wave speeds.  Speeds go stale only through set_state; after one
    // full step every problem that can still advance has the speeds of its
    // state (gathered by stage 3), so later steps use the lighter graph.
    hipGraphExec_t graph = nullptr, graph_fast = nullptr;
    hipGraph_t graph_def = nullptr, graph_fast_def = nullptr;
    int speeds_fresh = 0;
    // STEPS_PER_GRAPH lighter steps in one graph (hweno_steps, run_to_time):
    // kernels inside a graph follow each other without a gap, while separate
    // graph launches on a stream are several microseconds apart
    hipGraphExec_t graph_multi = nullptr;
    hipGraph_t graph_multi_def = nullptr;
    hweno_tuning tun{};
    Scheme sch{};
    std::string err;
};

static thread_local std::string g_create_error;

static int fail(hweno_handle* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_create_error = buf;
    return code;
}

#define HIP_TRY(h, call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((h), HWENO_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static int ncomp_of(const hweno_problem& p) {
    if (p.flux != HWENO_EULER) return 1;
    return p.dim == 1 ? 3 : 4;
}

static void prec_sizes(int prec, size_t* su, size_t* sd) {
    *su = prec == HWENO_F32 ? 4 : 8;   // F32_KAHAN keeps (hi, lo) float pairs
    *sd = prec == HWENO_F64 ? 8 : 4;
}

// Sizes of every region of a handle's workspace.
struct Layout {
    size_t u_bytes, d_bytes, probs, ctl, tiles, chunks, stage, total;
    size_t tiles_cap;
    int nchunks;
    size_t stage_elems;
};

static int tiles_2d(int nx, int ny, int rows) {
    return ((nx + STRIP_OUT - 1) / STRIP_OUT) * ((ny + rows - 1) / rows);
}

static int validate(const hweno_problem* probs, int32_t nprob, const hweno_config* cfg,
                    hweno_handle* h);

namespace hweno {
int validate_problems(const hweno_problem* probs, int32_t nprob, const hweno_config* cfg) {
    return validate(probs, nprob, cfg, nullptr);
}

int thread_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_create_error = buf;
    return code;
}

Scheme scheme_of(const hweno_problem& p0, const hweno_config& cfg) {
    Scheme s{};
    for (int m = 0; m < 5; ++m) s.gam[m] = cfg.gamma_lin[m];
    s.eps = cfg.eps;
    s.gas_gamma = p0.gas_gamma;
    s.adv[0] = p0.adv[0];
    s.adv[1] = p0.adv[1];
    s.weights = cfg.weights;
    s.Q = cfg.gauss_q;
    s.charwise = cfg.characteristic && p0.flux == F_EULER;
    s.smoothness = cfg.smoothness;
    return s;
}

ProbDev probdev_of(const hweno_problem& pr, const hweno_config& cfg, int64_t off_u,
                   int64_t off_d) {
    ProbDev d;
    std::memset(&d, 0, sizeof d);
    d.nx = pr.nx;
    d.ny = pr.ny;
    d.bc_x = pr.bc_x;
    d.bc_y = pr.dim == 2 ? pr.bc_y : HWENO_PERIODIC;
    d.off_u = off_u;
    d.off_d = off_d;
    d.dx = (pr.xhi - pr.xlo) / pr.nx;
    d.dy = pr.dim == 2 ? (pr.yhi - pr.ylo) / pr.ny : 1.0;
    d.inv_dx = 1.0 / d.dx;
    d.inv_dy = 1.0 / d.dy;
    d.dxe = std::pow(d.dx, cfg.dt_exponent);
    d.dye = std::pow(d.dy, cfg.dt_exponent);
    d.t = 0.0;
    d.t_end = pr.t_end;
    d.bad_cell = INT64_MAX;
    return d;
}
}  // namespace hweno

static int validate(const hweno_problem* probs, int32_t nprob, const hweno_config* cfg,
                    hweno_handle* h) {
    if (!probs || nprob <= 0 || !cfg) return fail(h, HWENO_ERR_ARG, "no problems or no config");
    const int dim = probs[0].dim, flux = probs[0].flux;
    if (dim != 1 && dim != 2) return fail(h, HWENO_ERR_ARG, "dim must be 1 or 2");
    if (flux < 0 || flux > 2) return fail(h, HWENO_ERR_ARG, "unknown flux family %d", flux);
    for (int p = 0; p < nprob; ++p) {
        const hweno_problem& q = probs[p];
        if (q.dim != dim || q.flux != flux)
            return fail(h, HWENO_ERR_ARG, "problem %d: dim/flux differ from problem 0", p);
        if (q.nx < 4) return fail(h, HWENO_ERR_ARG, "problem %d: nx < 4", p);
        if (dim == 1 && q.ny != 1) return fail(h, HWENO_ERR_ARG, "problem %d: ny must be 1 in 1D", p);
        if (dim == 2 && q.ny < 4) return fail(h, HWENO_ERR_ARG, "problem %d: ny < 4", p);
        if ((int64_t)q.nx * q.ny > (int64_t)INT32_MAX / 4)
            return fail(h, HWENO_ERR_ARG, "problem %d: too many cells", p);
        if (!(q.xhi > q.xlo) || (dim == 2 && !(q.yhi > q.ylo)))
            return fail(h, HWENO_ERR_ARG, "problem %d: empty domain", p);
        if (q.bc_x < HWENO_PERIODIC || q.bc_x > HWENO_REFLECTIVE ||
            (dim == 2 && (q.bc_y < HWENO_PERIODIC || q.bc_y > HWENO_REFLECTIVE)))
            return fail(h, HWENO_ERR_ARG, "problem %d: unknown boundary type", p);
        if (flux != HWENO_EULER &&
            (q.bc_x == HWENO_REFLECTIVE || (dim == 2 && q.bc_y == HWENO_REFLECTIVE)))
            return fail(h, HWENO_ERR_ARG, "problem %d: reflective walls need the Euler flux", p);
        if (flux == HWENO_EULER && !(q.gas_gamma > 1.0))
            return fail(h, HWENO_ERR_ARG, "problem %d: gas_gamma must exceed 1", p);
        if (q.gas_gamma != probs[0].gas_gamma || q.adv[0] != probs[0].adv[0] ||
            q.adv[1] != probs[0].adv[1])
            return fail(h, HWENO_ERR_ARG, "problem %d: gas_gamma/adv differ from problem 0", p);
    }
    if (cfg->precision < HWENO_F64 || cfg->precision > HWENO_F32_KAHAN)
        return fail(h, HWENO_ERR_ARG, "precision %d not supported", cfg->precision);
    if (dim == 2 && cfg->gauss_q != 2 && cfg->gauss_q != 3)
        return fail(h, HWENO_ERR_ARG, "gauss_q must be 2 or 3");
    if (cfg->weights < HWENO_W_PAPER || cfg->weights > HWENO_W_LINEAR)
        return fail(h, HWENO_ERR_ARG, "unknown weight form %d", cfg->weights);
    const int M = dim == 1 ? 2 : 4;
    double s = 0.0;
    for (int m = 0; m <= M; ++m) {
        if (!(cfg->gamma_lin[m] > 0.0))
            return fail(h, HWENO_ERR_ARG, "linear weight gamma_%d must be positive", m);
        s += cfg->gamma_lin[m];
    }
    if (std::fabs(s - 1.0) > 1e-12) return fail(h, HWENO_ERR_ARG, "linear weights must sum to 1");
    if (!(cfg->eps > 0.0)) return fail(h, HWENO_ERR_ARG, "eps must be positive");
    if (!(cfg->cfl > 0.0)) return fail(h, HWENO_ERR_ARG, "cfl must be positive");
    if (!(cfg->dt_exponent > 0.0)) return fail(h, HWENO_ERR_ARG, "dt_exponent must be positive");
    if (cfg->characteristic != 0 && cfg->characteristic != 1)
        return fail(h, HWENO_ERR_ARG, "characteristic must be 0 or 1");
    if (cfg->smoothness != HWENO_BETA_MOMENT && cfg->smoothness != HWENO_BETA_CLASSICAL)
        return fail(h, HWENO_ERR_ARG, "unknown smoothness indicator %d", cfg->smoothness);
    if (cfg->alpha_stage != 0 && cfg->alpha_stage != 1)
        return fail(h, HWENO_ERR_ARG, "alpha_stage must be 0 or 1");
    return HWENO_OK;
}

static Layout layout_of(const hweno_problem* probs, int32_t nprob, const hweno_config* cfg) {
    Layout L{};
    const int K = ncomp_of(probs[0]);
    const int D = probs[0].dim;
    const int nvar = 1 + D;
    size_t su, sd;
    prec_sizes(cfg->precision, &su, &sd);
    size_t nu = 0, nd = 0, maxst = 0, tiles = 0;
    int nch = 0;
    for (int p = 0; p < nprob; ++p) {
        const size_t nc = (size_t)probs[p].nx * probs[p].ny;
        nu += (size_t)K * nc;
        nd += (size_t)K * D * nc;
        maxst = std::max(maxst, (size_t)nvar * K * nc);
        if (D == 1) tiles += (probs[p].nx + TILE1D_OUT - 1) / TILE1D_OUT;
        else tiles += tiles_2d(probs[p].nx, probs[p].ny, 8);  // smallest segment height
        nch += (int)((nc + CHUNK_CELLS - 1) / CHUNK_CELLS);
    }
    L.u_bytes = align256(nu * su);
    L.d_bytes = align256(nd * sd);
    L.probs = align256(sizeof(ProbDev) * nprob);
    L.ctl = align256(sizeof(StepCtl));
    L.tiles_cap = 2 * tiles;
    L.tiles = align256(L.tiles_cap * (D == 1 ? sizeof(Tile1D) : sizeof(Tile2D)));
    L.nchunks = nch;
    L.chunks = align256(sizeof(Chunk) * nch);
    L.stage_elems = 2 * maxst;
    L.stage = align256(sizeof(double) * L.stage_elems);
    L.total = 3 * (L.u_bytes + L.d_bytes) + L.d_bytes + L.probs + L.ctl + L.tiles + L.chunks +
              L.stage;
    return L;
}

// ------------------------------------------------------------- work lists

// Builds the tile lists: the step list (all problems, neighbouring tiles
// grouped so that each of the eight XCDs of the GPU works on a contiguous
// region: list position 8k + x holds the k-th tile of region x, and the
// dispatcher hands workgroup b to XCD b mod 8), then the per-problem list.
static int build_tiles(hweno_handle* h) {
    const int rows = h->tun.tile_rows;
    std::vector<int> begin(h->nprob), count(h->nprob);
    if (h->dim == 1) {
        std::vector<Tile1D> per;
        for (int p = 0; p < h->nprob; ++p) {
            begin[p] = (int)per.size();
            for (int c0 = 0; c0 < h->probs[p].nx; c0 += TILE1D_OUT) per.push_back({p, c0});
            count[p] = (int)per.size() - begin[p];
        }
        const size_t n = per.size();
        if (2 * n > h->tiles_cap) return fail(h, HWENO_ERR_OOM, "tile list exceeds its buffer");
        std::vector<Tile1D> all(per);
        all.insert(all.end(), per.begin(), per.end());
        HIP_TRY(h, hipMemcpy(h->d_tiles, all.data(), all.size() * sizeof(Tile1D),
                             hipMemcpyHostToDevice));
        h->ntiles_step = (int)n;
        for (int& b : begin) b += (int)n;
    } else {
        std::vector<Tile2D> per;
        for (int p = 0; p < h->nprob; ++p) {
            begin[p] = (int)per.size();
            const int nx = h->probs[p].nx, ny = h->probs[p].ny;
            for (int j0 = 0; j0 < ny; j0 += rows)
                for (int i0 = 0; i0 < nx; i0 += STRIP_OUT)
                    per.push_back({p, i0, j0, std::min(rows, ny - j0)});
            count[p] = (int)per.size() - begin[p];
        }
        const size_t n = per.size();
        if (2 * n > h->tiles_cap) return fail(h, HWENO_ERR_OOM, "tile list exceeds its buffer");
        std::vector<Tile2D> step(n);
        const size_t nreg = 8;
        size_t pos = 0;
        // region x = contiguous slice [x*n/8, (x+1)*n/8) of the per-problem order
        std::vector<size_t> rb(nreg + 1);
        for (size_t x = 0; x <= nreg; ++x) rb[x] = x * n / nreg;
        for (size_t k = 0; pos < n; ++k)
            for (size_t x = 0; x < nreg; ++x)
                if (rb[x] + k < rb[x + 1]) step[pos++] = per[rb[x] + k];
        std::vector<Tile2D> all(step);
        all.insert(all.end(), per.begin(), per.end());
        HIP_TRY(h, hipMemcpy(h->d_tiles, all.data(), all.size() * sizeof(Tile2D),
                             hipMemcpyHostToDevice));
        h->ntiles_step = (int)n;
        for (int& b : begin) b += (int)n;
    }
    h->tile_begin = begin;
    h->tile_count = count;
    return HWENO_OK;
}

static void drop_graph(hweno_handle* h) {
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->graph_def) (void)hipGraphDestroy(h->graph_def);
    if (h->graph_fast) (void)hipGraphExecDestroy(h->graph_fast);
    if (h->graph_fast_def) (void)hipGraphDestroy(h->graph_fast_def);
    if (h->graph_multi) (void)hipGraphExecDestroy(h->graph_multi);
    if (h->graph_multi_def) (void)hipGraphDestroy(h->graph_multi_def);
    h->graph = h->graph_fast = h->graph_multi = nullptr;
    h->graph_def = h->graph_fast_def = h->graph_multi_def = nullptr;
}

// ----------------------------------------------------------------- create

extern "C" void hweno_default_config(int32_t dim, hweno_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->precision = HWENO_F64;
    cfg->gauss_q = 3;
    cfg->weights = HWENO_W_BETA;
    const int M = dim == 1 ? 2 : 4;
    cfg->gamma_lin[0] = 1.0 - M / 400.0;
    for (int m = 1; m <= M; ++m) cfg->gamma_lin[m] = 1.0 / 400.0;
    cfg->eps = 1e-8;
    cfg->cfl = 0.6;
    cfg->dt_exponent = 1.0;
}

extern "C" size_t hweno_workspace_bytes(const hweno_problem* probs, int32_t nprob,
                                        const hweno_config* cfg) {
    if (validate(probs, nprob, cfg, nullptr) != HWENO_OK) return 0;
    return layout_of(probs, nprob, cfg).total;
}

static int setup(hweno_handle* h, const hweno_problem* probs, int32_t nprob,
                 const hweno_config* cfg, void* workspace, size_t ws_bytes, void* stream) {
    h->cfg = *cfg;
    h->probs.assign(probs, probs + nprob);
    h->nprob = nprob;
    h->dim = probs[0].dim;
    h->flux = probs[0].flux;
    h->K = ncomp_of(probs[0]);
    h->D = h->dim;
    h->nvar = 1 + h->D;
    h->prec = cfg->precision;
    prec_sizes(h->prec, &h->su, &h->sd);
    const Layout L = layout_of(probs, nprob, cfg);
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        HIP_TRY(h, hipStreamCreate(&h->stream));
        h->own_stream = true;
    }
    if (workspace) {
        if (ws_bytes < L.total)
            return fail(h, HWENO_ERR_OOM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
        h->ws = (char*)workspace;
    } else {
        hipError_t e = hipMalloc((void**)&h->ws, L.total);
        if (e != hipSuccess)
            return fail(h, HWENO_ERR_OOM, "hipMalloc of %zu bytes failed: %s", L.total,
                        hipGetErrorString(e));
        h->own_ws = true;
    }
    h->ws_bytes = L.total;
    char* p = h->ws;
    for (int s = 0; s < 3; ++s) {
        h->U[s].u = p; p += L.u_bytes;
        h->U[s].d = p; p += L.d_bytes;
    }
    h->H = p; p += L.d_bytes;
    h->d_probs = (ProbDev*)p; p += L.probs;
    h->d_ctl = (StepCtl*)p; p += L.ctl;
    h->d_tiles = p; p += L.tiles;
    h->tiles_cap = L.tiles_cap;
    h->d_chunks = (Chunk*)p; p += L.chunks;
    h->d_stage = (double*)p; p += L.stage;
    h->stage_elems = L.stage_elems;
    h->nchunks = L.nchunks;

    h->sch = scheme_of(probs[0], *cfg);

    // problem table
    h->h_probs.resize(nprob);
    h->ncell.resize(nprob);
    int64_t ou = 0, od = 0;
    std::vector<Chunk> chunks;
    for (int q = 0; q < nprob; ++q) {
        const hweno_problem& pr = probs[q];
        h->h_probs[q] = probdev_of(pr, *cfg, ou, od);
        const int64_t nc = (int64_t)pr.nx * pr.ny;
        h->ncell[q] = nc;
        ou += (int64_t)h->K * nc;
        od += (int64_t)h->K * h->D * nc;
        for (int64_t s = 0; s < nc; s += CHUNK_CELLS)
            chunks.push_back({q, (int32_t)s, (int32_t)std::min<int64_t>(CHUNK_CELLS, nc - s), 0});
    }
    HIP_TRY(h, hipMemcpy(h->d_probs, h->h_probs.data(), sizeof(ProbDev) * nprob,
                         hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->d_chunks, chunks.data(), sizeof(Chunk) * chunks.size(),
                         hipMemcpyHostToDevice));
    StepCtl ctl{};
    ctl.cfl = cfg->cfl;
    ctl.nprob = nprob;
    ctl.dim = h->dim;
    HIP_TRY(h, hipMemcpy(h->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice));
    h->state_set.assign(nprob, 0);
    h->tun.tile_rows = 32;
    h->tun.grid_blocks = 0;
    h->tun.use_graph = 1;
    h->tun.variant = 0;
    h->tun.source = HWENO_TUNED_DEFAULT;
    return build_tiles(h);
}

extern "C" int hweno_create(const hweno_problem* probs, int32_t nprob, const hweno_config* cfg,
                            void* workspace, size_t ws_bytes, void* hip_stream,
                            hweno_handle** out) {
    if (!out) return fail(nullptr, HWENO_ERR_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate(probs, nprob, cfg, nullptr);
    if (rc) return rc;
    hweno_handle* h = new hweno_handle();
    rc = setup(h, probs, nprob, cfg, workspace, ws_bytes, hip_stream);
    if (rc) {
        g_create_error = h->err;
        hweno_destroy(h);
        return rc;
    }
    *out = h;
    return HWENO_OK;
}

extern "C" int hweno_destroy(hweno_handle* h) {
    if (!h) return HWENO_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return HWENO_OK;
}

extern "C" const char* hweno_last_error(const hweno_handle* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

// ------------------------------------------------------------ device table

static int read_probs(hweno_handle* h, std::vector<ProbDev>& v) {
    v.resize(h->nprob);
    HIP_TRY(h, hipMemcpyAsync(v.data(), h->d_probs, sizeof(ProbDev) * h->nprob,
                              hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return HWENO_OK;
}

static int report_errors(hweno_handle* h, const std::vector<ProbDev>& v, int only = -1) {
    for (int p = 0; p < h->nprob; ++p) {
        if (only >= 0 && p != only) continue;
        if (v[p].err) {
            const int64_t c = v[p].bad_cell;
            const int nx = v[p].nx;
            return fail(h, HWENO_ERR_NONFINITE,
                        "problem %d: non-admissible state (non-finite, or rho <= 0 / p <= 0) "
                        "at cell i=%lld j=%lld, t=%.17g",
                        p, (long long)(c % nx), (long long)(c / nx), v[p].t);
        }
    }
    return HWENO_OK;
}

static int check_prob(hweno_handle* h, int32_t prob) {
    if (!h) return HWENO_ERR_ARG;
    if (prob < 0 || prob >= h->nprob)
        return fail(h, HWENO_ERR_ARG, "problem index %d out of range [0, %d)", prob, h->nprob);
    return HWENO_OK;
}

extern "C" int hweno_set_state(hweno_handle* h, int32_t prob, const double* src,
                               int32_t src_on_device, double t) {
    int rc = check_prob(h, prob);
    if (rc) return rc;
    if (!src) return fail(h, HWENO_ERR_ARG, "src is NULL");
    const int64_t n = (int64_t)h->nvar * h->K * h->ncell[prob];
    HIP_TRY(h, hipMemcpyAsync(h->d_stage, src, sizeof(double) * n,
                              src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              h->stream));
    HIP_TRY(h, launch_pack(h->prec, 1, h->d_stage, h->U[0], h->h_probs[prob].off_u,
                           h->h_probs[prob].off_d, h->K, h->nvar, h->ncell[prob], h->stream));
    ProbDev d;
    HIP_TRY(h, hipMemcpyAsync(&d, h->d_probs + prob, sizeof d, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    d.t = t;
    d.err = 0;
    d.bad_cell = INT64_MAX;
    d.active = 0;
    d.alpha_valid = 0;
    HIP_TRY(h, hipMemcpyAsync(h->d_probs + prob, &d, sizeof d, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->state_set[prob] = 1;
    h->speeds_fresh = 0;
    return HWENO_OK;
}

extern "C" int hweno_get_state(hweno_handle* h, int32_t prob, double* dst,
                               int32_t dst_on_device, double* t) {
    int rc = check_prob(h, prob);
    if (rc) return rc;
    if (!h->state_set[prob]) return fail(h, HWENO_ERR_STATE, "problem %d has no state yet", prob);
    const int64_t n = (int64_t)h->nvar * h->K * h->ncell[prob];
    std::vector<ProbDev> v(h->nprob);
    HIP_TRY(h, hipMemcpyAsync(&v[prob], h->d_probs + prob, sizeof(ProbDev), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (dst) {
        HIP_TRY(h, launch_pack(h->prec, 0, h->d_stage, h->U[0], h->h_probs[prob].off_u,
                               h->h_probs[prob].off_d, h->K, h->nvar, h->ncell[prob], h->stream));
        HIP_TRY(h, hipMemcpyAsync(dst, h->d_stage, sizeof(double) * n,
                                  dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    if (t) *t = v[prob].t;
    return report_errors(h, v, prob);
}

extern "C" int hweno_sync(hweno_handle* h) {
    if (!h) return HWENO_ERR_ARG;
    std::vector<ProbDev> v;
    int rc = read_probs(h, v);
    if (rc) return rc;
    return report_errors(h, v);
}

// ------------------------------------------------------------- operators

static StageArgs stage_args(hweno_handle* h, int mode) {
    StageArgs a{};
    const int k = mode == MODE_RHS ? 0 : mode - 1;  // input set of the stage
    a.in = h->U[k];
    a.out = h->U[mode == MODE_S3 ? 0 : (k + 1) % 3];
    a.un = h->U[0].u;
    a.h = h->H;
    a.probs = h->d_probs;
    a.tiles = h->d_tiles;
    a.ntiles = h->ntiles_step;
    a.tile_offset = 0;
    a.sch = h->sch;
    return a;
}

static hipError_t launch_stage(hweno_handle* h, int mode, const StageArgs& a) {
    if (h->dim == 1) return launch_stage1d(h->prec, h->flux, mode, a, h->tun.grid_blocks, h->stream);
    return launch_stage2d(h->prec, h->flux, h->cfg.gauss_q, mode, h->tun.variant, a,
                          h->tun.grid_blocks, h->stream);
}

static int alpha_all(hweno_handle* h) {
    HIP_TRY(h, launch_reset(h->d_probs, h->d_ctl, h->nprob, SEL_ALL, h->stream));
    HIP_TRY(h, launch_alpha(h->prec, h->flux, h->dim, h->U[0].u, h->d_probs, h->d_chunks,
                            h->nchunks, h->sch, SEL_ALL, 0, h->stream));
    return HWENO_OK;
}

extern "C" int hweno_alpha(hweno_handle* h, int32_t prob, double* ax, double* ay) {
    int rc = check_prob(h, prob);
    if (rc) return rc;
    if (!h->state_set[prob]) return fail(h, HWENO_ERR_STATE, "problem %d has no state yet", prob);
    rc = alpha_all(h);
    if (rc) return rc;
    std::vector<ProbDev> v;
    rc = read_probs(h, v);
    if (rc) return rc;
    double x, y;
    std::memcpy(&x, &v[prob].ax_bits, 8);
    std::memcpy(&y, &v[prob].ay_bits, 8);
    if (ax) *ax = x;
    if (ay) *ay = y;
    return report_errors(h, v, prob);
}

extern "C" int hweno_rhs(hweno_handle* h, int32_t prob, double* L_out, double* Uhat_out,
                         int32_t on_device) {
    int rc = check_prob(h, prob);
    if (rc) return rc;
    if (!h->state_set[prob]) return fail(h, HWENO_ERR_STATE, "problem %d has no state yet", prob);
    // the 2D rhs uses the per-problem tiles of the current tiling
    rc = alpha_all(h);
    if (rc) return rc;
    const int64_t n = (int64_t)h->nvar * h->K * h->ncell[prob];
    StageArgs a = stage_args(h, MODE_RHS);
    a.L_out = (on_device && L_out) ? L_out : h->d_stage;
    a.Uh_out = (on_device && Uhat_out) ? Uhat_out : h->d_stage + n;
    a.tile_offset = h->tile_begin[prob];
    a.ntiles = h->tile_count[prob];
    HIP_TRY(h, launch_stage(h, MODE_RHS, a));
    if (!on_device) {
        if (L_out)
            HIP_TRY(h, hipMemcpyAsync(L_out, a.L_out, sizeof(double) * n, hipMemcpyDeviceToHost,
                                      h->stream));
        if (Uhat_out)
            HIP_TRY(h, hipMemcpyAsync(Uhat_out, a.Uh_out, sizeof(double) * n,
                                      hipMemcpyDeviceToHost, h->stream));
    }
    std::vector<ProbDev> v;
    rc = read_probs(h, v);
    if (rc) return rc;
    return report_errors(h, v, prob);
}

// One SSP-RK3 step of every unfinished problem: wave speeds and dt, three
// fused stage kernels, time update.
// The launches of one step, in order; rec(kind, launch) issues each one
// (and may bracket it with events).
enum LaunchKind { LK_OTHER = 0, LK_ALPHA = 1, LK_STAGE = 2 };

// One step.  fast: no problem that can advance has stale speeds, so the
// reduction kernel is left out (and with at most 256 problems the dt kernel
// clears the step counters itself, which leaves out the reset kernel too).
template <class Rec>
static int enqueue_step_with(hweno_handle* h, int use_dt_in, bool fast, Rec&& rec) {
    const int own_ctl = fast && h->nprob <= 256;
    // speeds are gathered by stage 3 of the previous step; the reduction
    // kernel only fills them in after set_state
    if (!own_ctl)
        HIP_TRY(h, rec(LK_OTHER, [&] { return launch_reset(h->d_probs, h->d_ctl, h->nprob, SEL_STALE, h->stream); }));
    if (!fast)
        HIP_TRY(h, rec(LK_ALPHA, [&] {
            return launch_alpha(h->prec, h->flux, h->dim, h->U[0].u, h->d_probs, h->d_chunks,
                                h->nchunks, h->sch, SEL_STALE, 0, h->stream);
        }));
    HIP_TRY(h, rec(LK_OTHER, [&] { return launch_dt(h->d_probs, h->d_ctl, h->nprob, use_dt_in, own_ctl, h->stream); }));
    for (int mode = MODE_S1; mode <= MODE_S3; ++mode) {
        if (mode != MODE_S1 && h->cfg.alpha_stage) {
            // speeds of this stage's input (per-stage option)
            const void* uin = h->U[mode - 1].u;
            HIP_TRY(h, rec(LK_OTHER, [&] { return launch_reset(h->d_probs, h->d_ctl, h->nprob, SEL_ACTIVE, h->stream); }));
            HIP_TRY(h, rec(LK_ALPHA, [&] {
                return launch_alpha(h->prec, h->flux, h->dim, uin, h->d_probs, h->d_chunks,
                                    h->nchunks, h->sch, SEL_ACTIVE, 0, h->stream);
            }));
        }
        HIP_TRY(h, rec(LK_STAGE, [&] { return launch_stage(h, mode, stage_args(h, mode)); }));
    }
    HIP_TRY(h, rec(LK_OTHER, [&] { return launch_finish(h->d_probs, h->d_ctl, h->nprob, h->stream); }));
    return HWENO_OK;
}

static int enqueue_step(hweno_handle* h, int use_dt_in, bool fast) {
    int rc = enqueue_step_with(h, use_dt_in, fast, [](int, auto&& launch) { return launch(); });
    if (rc == HWENO_OK) h->speeds_fresh = 1;
    return rc;
}

static int launch_step(hweno_handle* h) {
    const bool fast = h->speeds_fresh != 0;
    if (!h->tun.use_graph) return enqueue_step(h, 0, fast);
    hipGraphExec_t& exec = fast ? h->graph_fast : h->graph;
    hipGraph_t& def = fast ? h->graph_fast_def : h->graph_def;
    if (!exec) {
        HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_step_with(h, 0, fast, [](int, auto&& launch) { return launch(); });
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(h->stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess)
            return fail(h, HWENO_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        def = g;
        HIP_TRY(h, hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
    }
    HIP_TRY(h, hipGraphLaunch(exec, h->stream));
    h->speeds_fresh = 1;
    return HWENO_OK;
}

constexpr int STEPS_PER_GRAPH = 8;

// Captures STEPS_PER_GRAPH lighter steps as one graph (speeds must be current).
static int capture_multi(hweno_handle* h) {
    HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = HWENO_OK;
    for (int k = 0; k < STEPS_PER_GRAPH && rc == HWENO_OK; ++k)
        rc = enqueue_step_with(h, 0, true, [](int, auto&& launch) { return launch(); });
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(h, HWENO_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    h->graph_multi_def = g;
    HIP_TRY(h, hipGraphInstantiate(&h->graph_multi, g, nullptr, nullptr, 0));
    return HWENO_OK;
}

// n steps with the CFL rule, enqueued: the first step after set_state alone,
// then whole graphs of STEPS_PER_GRAPH steps, then single steps.  In graph
// mode the multi-step graph is built as soon as the speeds are current, also
// when n does not reach it, so that a warm-up call leaves nothing to build.
static int launch_steps(hweno_handle* h, int64_t n) {
    int64_t done = 0;
    int rc = HWENO_OK;
    if (!h->tun.use_graph) {
        for (; done < n && rc == HWENO_OK; ++done) rc = launch_step(h);
        return rc;
    }
    if (n > 0 && !h->speeds_fresh) {
        rc = launch_step(h);
        if (rc) return rc;
        ++done;
    }
    if (h->speeds_fresh && !h->graph_multi) {
        rc = capture_multi(h);
        if (rc) return rc;
    }
    for (; n - done >= STEPS_PER_GRAPH; done += STEPS_PER_GRAPH)
        HIP_TRY(h, hipGraphLaunch(h->graph_multi, h->stream));
    for (; done < n && rc == HWENO_OK; ++done) rc = launch_step(h);
    return rc;
}

static int all_set(hweno_handle* h) {
    for (int p = 0; p < h->nprob; ++p)
        if (!h->state_set[p]) return fail(h, HWENO_ERR_STATE, "problem %d has no state yet", p);
    return HWENO_OK;
}

extern "C" int hweno_step(hweno_handle* h, const double* dt_in, double* dt_out) {
    if (!h) return HWENO_ERR_ARG;
    int rc = all_set(h);
    if (rc) return rc;
    if (dt_in) {
        std::vector<ProbDev> v;
        rc = read_probs(h, v);
        if (rc) return rc;
        for (int p = 0; p < h->nprob; ++p) v[p].dt_in = dt_in[p];
        HIP_TRY(h, hipMemcpyAsync(h->d_probs, v.data(), sizeof(ProbDev) * h->nprob,
                                  hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        rc = enqueue_step(h, 1, h->speeds_fresh != 0);
    } else {
        rc = launch_step(h);
    }
    if (rc) return rc;
    if (dt_out) {
        std::vector<ProbDev> v;
        rc = read_probs(h, v);
        if (rc) return rc;
        for (int p = 0; p < h->nprob; ++p) dt_out[p] = v[p].active ? v[p].dt : 0.0;
        return report_errors(h, v);
    }
    return HWENO_OK;
}

extern "C" int hweno_steps(hweno_handle* h, int32_t nsteps) {
    if (!h) return HWENO_ERR_ARG;
    if (nsteps < 0) return fail(h, HWENO_ERR_ARG, "nsteps must be >= 0");
    int rc = all_set(h);
    if (rc) return rc;
    return launch_steps(h, nsteps);
}

extern "C" int hweno_run_to_time(hweno_handle* h, int64_t* steps_out) {
    if (!h) return HWENO_ERR_ARG;
    int rc = all_set(h);
    if (rc) return rc;
    StepCtl ctl{};
    HIP_TRY(h, hipMemcpyAsync(&ctl, h->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const int64_t steps0 = ctl.steps;
    int batch = 4;
    for (;;) {
        rc = launch_steps(h, batch);
        if (rc) return rc;
        HIP_TRY(h, hipMemcpyAsync(&ctl, h->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        if (ctl.nactive == 0) break;
        batch = std::min(batch * 2, 64);
    }
    if (steps_out) *steps_out = ctl.steps - steps0;
    return hweno_sync(h);
}

// ----------------------------------------------------------------- tuning

extern "C" int hweno_get_tuning(const hweno_handle* h, hweno_tuning* t) {
    if (!h || !t) return HWENO_ERR_ARG;
    *t = h->tun;
    return HWENO_OK;
}

static int apply_tuning(hweno_handle* h, const hweno_tuning* t, int source) {
    if (t->tile_rows < 8 || t->tile_rows > 1024)
        return fail(h, HWENO_ERR_ARG, "tile_rows must lie in [8, 1024]");
    if (t->grid_blocks < 0) return fail(h, HWENO_ERR_ARG, "grid_blocks must be >= 0");
    if (t->use_graph != 0 && t->use_graph != 1) return fail(h, HWENO_ERR_ARG, "use_graph must be 0 or 1");
    if (t->variant != 0 && t->variant != 1) return fail(h, HWENO_ERR_ARG, "variant must be 0 or 1");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    drop_graph(h);
    h->tun = *t;
    h->tun.source = source;
    return build_tiles(h);
}

extern "C" int hweno_set_tuning(hweno_handle* h, const hweno_tuning* t) {
    if (!h || !t) return HWENO_ERR_ARG;
    return apply_tuning(h, t, HWENO_TUNED_BY_CALLER);
}

// Tuning cache: one JSON object per line,
//   {"key": "<arch>|cu<n>|dim<d>|flux<f>|prec<p>|q<Q>|char<c>|p2^<a>|c2^<b>",
//    "tile_rows": r, "grid_blocks": g, "variant": v, "step_ms": t}
// (problems and cells rounded to powers of two); the last line with a key wins.
static std::string tuning_key(hweno_handle* h) {
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
        ncu = prop.multiProcessorCount;
    }
    int64_t cells = 0;
    for (int64_t c : h->ncell) cells += c;
    auto lg = [](double x) { return (int)std::lround(std::log2(std::max(1.0, x))); };
    char buf[256];
    snprintf(buf, sizeof buf, "%s|cu%d|dim%d|flux%d|prec%d|q%d|char%d|p2^%d|c2^%d", arch.c_str(), ncu,
             h->dim, h->flux, h->prec, h->dim == 2 ? h->cfg.gauss_q : 0, h->sch.charwise,
             lg((double)h->nprob), lg((double)cells));
    return buf;
}

static bool cache_lookup(const char* path, const std::string& key, hweno_tuning* t) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    const std::string want = "\"key\": \"" + key + "\"";
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, want.c_str())) continue;
        int r = 0, g = 0, v = 0;
        const char* pr = std::strstr(line, "\"tile_rows\":");
        const char* pg = std::strstr(line, "\"grid_blocks\":");
        const char* pv = std::strstr(line, "\"variant\":");
        if (pr && pg && pv && std::sscanf(pr, "\"tile_rows\": %d", &r) == 1 &&
            std::sscanf(pg, "\"grid_blocks\": %d", &g) == 1 &&
            std::sscanf(pv, "\"variant\": %d", &v) == 1 && r >= 8 && r <= 1024 && g >= 0 &&
            (v == 0 || v == 1)) {
            t->tile_rows = r;
            t->grid_blocks = g;
            t->variant = v;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void cache_store(const char* path, const std::string& key, const hweno_tuning& t,
                        double ms) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;   // a cache that cannot be written is not an error
    std::fprintf(f,
                 "{\"key\": \"%s\", \"tile_rows\": %d, \"grid_blocks\": %d, \"variant\": %d, "
                 "\"step_ms\": %.6f}\n",
                 key.c_str(), t.tile_rows, t.grid_blocks, t.variant, ms);
    std::fclose(f);
}

// The launch configurations the tuner times.  2D: segment heights (the halo
// rows recomputed per segment against the number of workgroups), one
// workgroup per tile or a persistent grid of 2-4 per CU, and for the Euler
// kernels both register variants.  1D: tiles are fixed by the kernel; one
// workgroup per tile or a persistent grid.
static std::vector<hweno_tuning> tuning_candidates(hweno_handle* h) {
    std::vector<hweno_tuning> cands;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int graph = h->tun.use_graph;
    if (h->dim == 1) {
        for (int g : {0, 2 * ncu, 4 * ncu, 8 * ncu}) cands.push_back({64, g, graph, 0, 0, 0});
        return cands;
    }
    const int nvar = (h->flux == F_EULER && !h->sch.charwise) ? 2 : 1;
    for (int v = 0; v < nvar; ++v)
        for (int rows : {16, 24, 32, 48, 64})
            for (int g : {0, 2 * ncu, 3 * ncu, 4 * ncu}) cands.push_back({rows, g, graph, v, 0, 0});
    // With one workgroup per tile, a tile count just above a whole number of
    // rounds of the GPU's workgroup slots leaves a last round that runs the
    // chip mostly idle.  Also try the lowest segment heights whose tile count
    // fits 2 or 3 rounds at 3 or 4 resident workgroups per CU (the Euler
    // kernels' occupancy in double and single precision).
    auto ntiles = [&](int rows) {
        long long n = 0;
        for (const hweno_problem& p : h->probs)
            n += (long long)((p.nx + STRIP_OUT - 1) / STRIP_OUT) * ((p.ny + rows - 1) / rows);
        return n;
    };
    std::vector<int> fit;
    for (int per_cu : {3, 4})
        for (int rounds : {2, 3}) {
            const long long slots = (long long)rounds * per_cu * ncu;
            for (int rows = 16; rows <= 64; ++rows)
                if (ntiles(rows) <= slots) {
                    if (rows % 8 != 0 && std::find(fit.begin(), fit.end(), rows) == fit.end())
                        fit.push_back(rows);
                    break;
                }
        }
    for (int v = 0; v < nvar; ++v)
        for (int rows : fit) cands.push_back({rows, 0, graph, v, 0, 0});
    return cands;
}

// The candidate list hweno_autotune times, for callers that time or profile
// the candidates themselves.
extern "C" int hweno_tuning_candidates(hweno_handle* h, hweno_tuning* out, int32_t cap,
                                       int32_t* count) {
    if (!h || !count || cap < 0 || (cap > 0 && !out)) return HWENO_ERR_ARG;
    const std::vector<hweno_tuning> c = tuning_candidates(h);
    *count = (int32_t)c.size();
    for (int32_t i = 0; i < cap && i < (int32_t)c.size(); ++i) out[i] = c[i];
    return HWENO_OK;
}

// Times a few steps per candidate launch configuration from the same saved
// state and keeps the fastest; the state, times and counters are restored
// afterwards.  With HWENO_TUNING_CACHE naming a file, a configuration stored
// there for the same key is taken without timing, and a timed winner is
// appended to it.
extern "C" int hweno_autotune(hweno_handle* h, hweno_tuning* best) {
    if (!h) return HWENO_ERR_ARG;
    int rc = all_set(h);
    if (rc) return rc;
    const char* cache = std::getenv("HWENO_TUNING_CACHE");
    const std::string key = tuning_key(h);
    if (cache && *cache) {
        hweno_tuning t = h->tun;
        if (cache_lookup(cache, key, &t)) {
            rc = apply_tuning(h, &t, HWENO_TUNED_FROM_CACHE);
            if (rc) return rc;
            if (best) *best = h->tun;
            return HWENO_OK;
        }
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    std::vector<ProbDev> saved_probs;
    rc = read_probs(h, saved_probs);
    if (rc) return rc;
    StepCtl saved_ctl{};
    HIP_TRY(h, hipMemcpy(&saved_ctl, h->d_ctl, sizeof saved_ctl, hipMemcpyDeviceToHost));
    const int saved_fresh = h->speeds_fresh;
    const size_t ub = (size_t)((char*)h->U[0].d - (char*)h->U[0].u);
    const size_t db = (size_t)((char*)h->U[1].u - (char*)h->U[0].d);
    void* save = nullptr;
    HIP_TRY(h, hipMalloc(&save, ub + db));
    auto restore = [&]() -> int {
        HIP_TRY(h, hipMemcpyAsync(h->U[0].u, save, ub + db, hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(h, hipMemcpyAsync(h->d_probs, saved_probs.data(), sizeof(ProbDev) * h->nprob,
                                  hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipMemcpyAsync(h->d_ctl, &saved_ctl, sizeof saved_ctl, hipMemcpyHostToDevice,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        h->speeds_fresh = saved_fresh;   // the restored table may hold stale speeds
        return HWENO_OK;
    };
    HIP_TRY(h, hipMemcpyAsync(save, h->U[0].u, ub + db, hipMemcpyDeviceToDevice, h->stream));
    const std::vector<hweno_tuning> cands = tuning_candidates(h);
    const hweno_tuning keep = h->tun;
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    // GPU time of `nsteps` steps of candidate c after one untimed step (which
    // also builds its graphs), from the saved state; the state is restored
    auto time_cand = [&](const hweno_tuning& c, int nsteps, double* ms_out) -> int {
        int r = apply_tuning(h, &c, HWENO_TUNED_BY_TIMING);
        if (r) return r;
        r = launch_step(h);
        if (r) return r;
        HIP_TRY(h, hipEventRecord(e0, h->stream));
        for (int k = 0; k < nsteps && r == 0; ++k) r = launch_step(h);
        HIP_TRY(h, hipEventRecord(e1, h->stream));
        HIP_TRY(h, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
        if (r) return r;
        *ms_out = ms / nsteps;
        return restore();
    };
    // The clocks of an idle GPU ramp up only under load: steps of the first
    // candidate for at least 50 ms of GPU time before anything is compared.
    double warm_ms = 0.0;
    for (int k = 0; k < 64 && rc == 0 && warm_ms < 50.0; ++k) {
        double ms = 0.0;
        rc = time_cand(cands[0], 4, &ms);
        warm_ms += 5.0 * ms;
    }
    // Round 1: every candidate on three steps.  Round 2: the four fastest
    // and the configuration in use before, on six steps each, in two passes
    // in opposite orders, each keeping its lower time.  The configuration in
    // use before is kept unless another is more than 1% faster.
    std::vector<std::pair<double, size_t>> r1;
    for (size_t i = 0; i < cands.size() && rc == 0; ++i) {
        double ms = 0.0;
        rc = time_cand(cands[i], 3, &ms);
        r1.push_back({ms, i});
    }
    std::vector<hweno_tuning> fin;
    std::vector<double> fin_ms;
    if (rc == 0) {
        std::sort(r1.begin(), r1.end());
        fin.push_back(keep);
        for (size_t i = 0; i < r1.size() && fin.size() < 5; ++i) {
            const hweno_tuning& c = cands[r1[i].second];
            if (c.tile_rows == keep.tile_rows && c.grid_blocks == keep.grid_blocks &&
                c.variant == keep.variant)
                continue;
            fin.push_back(c);
        }
        fin_ms.assign(fin.size(), 1e300);
        for (int pass = 0; pass < 2 && rc == 0; ++pass)
            for (size_t n = 0; n < fin.size() && rc == 0; ++n) {
                const size_t i = pass ? fin.size() - 1 - n : n;
                double ms = 0.0;
                rc = time_cand(fin[i], 6, &ms);
                fin_ms[i] = std::min(fin_ms[i], ms);
            }
    }
    hweno_tuning win = keep;
    double best_ms = 1e300;
    if (rc == 0) {
        size_t b = 0;
        for (size_t i = 1; i < fin.size(); ++i)
            if (fin_ms[i] < fin_ms[b]) b = i;
        if (fin_ms[0] <= 1.01 * fin_ms[b]) b = 0;
        win = fin[b];
        best_ms = fin_ms[b];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int rc2 = restore();
    (void)hipFree(save);
    if (rc) {
        apply_tuning(h, &keep, keep.source);
        return rc;
    }
    if (rc2) return rc2;
    rc = apply_tuning(h, &win, HWENO_TUNED_BY_TIMING);
    if (rc) return rc;
    if (cache && *cache) cache_store(cache, key, win, best_ms);
    if (best) *best = h->tun;
    return HWENO_OK;
}

// ---------------------------------------------------------------- timing

extern "C" int hweno_timed_steps(hweno_handle* h, int32_t nsteps, hweno_timing* out) {
    if (!h || !out || nsteps < 0) return HWENO_ERR_ARG;
    int rc = all_set(h);
    if (rc) return rc;
    std::memset(out, 0, sizeof *out);
    // an event pair around every launch of every step
    std::vector<hipEvent_t> ev;
    std::vector<int> kinds;
    auto fresh = [&]() -> hipEvent_t {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ev.push_back(e);
        return e;
    };
    StepCtl c0{}, c1{};
    HIP_TRY(h, hipMemcpyAsync(&c0, h->d_ctl, sizeof c0, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    hipEvent_t start = fresh();
    if (!start) return fail(h, HWENO_ERR_HIP, "event creation failed");
    HIP_TRY(h, hipEventRecord(start, h->stream));
    for (int s = 0; s < nsteps && rc == HWENO_OK; ++s) {
        const bool fast = h->speeds_fresh != 0;
        rc = enqueue_step_with(h, 0, fast, [&](int kind, auto&& launch) -> hipError_t {
            hipEvent_t a = fresh(), b = fresh();
            if (!a || !b) return hipErrorOutOfMemory;
            hipError_t e = hipEventRecord(a, h->stream);
            if (e != hipSuccess) return e;
            e = launch();
            if (e != hipSuccess) return e;
            kinds.push_back(kind);
            return hipEventRecord(b, h->stream);
        });
        if (rc == HWENO_OK) h->speeds_fresh = 1;
    }
    hipEvent_t stop = rc == HWENO_OK ? fresh() : nullptr;
    if (stop) {
        HIP_TRY(h, hipEventRecord(stop, h->stream));
        HIP_TRY(h, hipEventSynchronize(stop));
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, start, stop));
        out->total_ms = ms;
        for (size_t i = 0; i < kinds.size(); ++i) {
            HIP_TRY(h, hipEventElapsedTime(&ms, ev[1 + 2 * i], ev[2 + 2 * i]));
            if (kinds[i] == LK_STAGE) {
                out->stage_ms += ms;
                out->stage_launches += 1;
            } else if (kinds[i] == LK_ALPHA) {
                out->alpha_ms += ms;
            } else {
                out->other_ms += ms;
            }
        }
    } else if (rc == HWENO_OK) {
        rc = fail(h, HWENO_ERR_HIP, "event creation failed");
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (rc) return rc;
    HIP_TRY(h, hipMemcpyAsync(&c1, h->d_ctl, sizeof c1, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out->steps = c1.steps - c0.steps;
    return hweno_sync(h);
}
