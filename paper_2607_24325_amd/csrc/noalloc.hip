// Allocation-free single-problem step (hweno_step_noalloc): the kernels of
// hweno_step, with every intermediate buffer (stage states, saved hats,
// problem table, step control, tile and reduction lists) in one fixed device
// array instead of a handle's workspace.  Nothing is allocated and nothing is
// copied between host and device: the problem table and work lists are
// written by a set-up kernel from launch arguments, so the whole call is a
// sequence of kernel launches on the caller's stream.
#include <algorithm>
#include <mutex>

#include "internal.h"

namespace hweno {

// The scratch of the allocation-free step: one copy per GPU, present from the
// library's first use on that GPU until the process ends.  In host code this
// name is only a stand-in; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[HWENO_NOALLOC_SCRATCH_BYTES];

// Writes the table entry, the step control, the tile list and the reduction
// chunks of one problem into the scratch (per-problem order; results do not
// depend on the order of the tiles).
__global__ void noalloc_setup_kernel(ProbDev pd, StepCtl ctl, ProbDev* probs, StepCtl* dctl,
                                     int dim, int rows, void* tiles, int ntiles, Chunk* chunks,
                                     int nchunks) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    if (tid == 0) {
        *probs = pd;
        *dctl = ctl;
    }
    const int strips = (pd.nx + STRIP_OUT - 1) / STRIP_OUT;
    for (int t = tid; t < ntiles; t += nth) {
        if (dim == 1) {
            ((Tile1D*)tiles)[t] = Tile1D{0, t * TILE1D_OUT};
        } else {
            const int js = t / strips, is = t - js * strips;
            const int j0 = js * rows;
            ((Tile2D*)tiles)[t] = Tile2D{0, is * STRIP_OUT, j0, min(rows, pd.ny - j0)};
        }
    }
    const int64_t nc = (int64_t)pd.nx * pd.ny;
    for (int k = tid; k < nchunks; k += nth) {
        const int64_t s0 = (int64_t)k * CHUNK_CELLS;
        const int64_t cnt = nc - s0 < CHUNK_CELLS ? nc - s0 : CHUNK_CELLS;
        chunks[k] = Chunk{0, (int32_t)s0, (int32_t)cnt, 0};
    }
}

// The step taken (0 if none) and the first non-admissible cell (-1 if none).
__global__ void noalloc_report_kernel(const ProbDev* probs, double* dt_out, int64_t* bad_out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const ProbDev P = *probs;
    if (dt_out) *dt_out = (P.active && !P.err) ? P.dt : 0.0;
    if (bad_out) *bad_out = P.err ? P.bad_cell : -1;
}

static std::mutex g_mu;
constexpr int MAX_DEVICES = 64;
static void* g_scratch[MAX_DEVICES];   // device address of `scratch`, per device

// Device address of the current device's scratch, looked up once per device.
static int scratch_address(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return thread_error(HWENO_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES)
        return thread_error(HWENO_ERR_HIP, "device %d beyond the %d the step supports", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return thread_error(HWENO_ERR_HIP, "hipGetSymbolAddress of the scratch failed: %s",
                                hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = (char*)g_scratch[dev];
    return HWENO_OK;
}

static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace hweno

using namespace hweno;

#define NA_TRY(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return thread_error(HWENO_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

extern "C" int hweno_step_noalloc(const hweno_problem* prob, const hweno_config* cfg,
                                  const double* state_in, double* state_out, double t,
                                  double dt_in, double* dt_out, int64_t* bad_out,
                                  void* hip_stream) {
    int rc = validate_problems(prob, 1, cfg);
    if (rc) return rc;
    if (!state_in || !state_out) return thread_error(HWENO_ERR_ARG, "state_in/state_out is NULL");
    const hweno_problem& pr = *prob;
    const int dim = pr.dim, flux = pr.flux, prec = cfg->precision;
    const int K = flux == HWENO_EULER ? (dim == 1 ? 3 : 4) : 1;
    const int D = dim, nvar = 1 + D;
    const size_t su = prec == HWENO_F32 ? 4 : 8, sd = prec == HWENO_F64 ? 8 : 4;
    const int64_t ncell = (int64_t)pr.nx * pr.ny;
    const int rows = 32;
    const int ntiles = dim == 1 ? (pr.nx + TILE1D_OUT - 1) / TILE1D_OUT
                                : ((pr.nx + STRIP_OUT - 1) / STRIP_OUT) * ((pr.ny + rows - 1) / rows);
    const int nchunks = (int)((ncell + CHUNK_CELLS - 1) / CHUNK_CELLS);
    // regions: three state sets, the saved hats, table, control, tiles, chunks
    const size_t ub = up256((size_t)ncell * K * su), db = up256((size_t)ncell * K * D * sd);
    const size_t tb = up256((size_t)ntiles * (dim == 1 ? sizeof(Tile1D) : sizeof(Tile2D)));
    const size_t cb = up256((size_t)nchunks * sizeof(Chunk));
    const size_t need = 3 * (ub + db) + db + up256(sizeof(ProbDev)) + up256(sizeof(StepCtl)) + tb + cb;
    if (need > HWENO_NOALLOC_SCRATCH_BYTES)
        return thread_error(HWENO_ERR_ARG,
                            "problem of %lld cells needs %zu bytes of scratch; the allocation-free "
                            "step has %zu (use a handle for larger problems)",
                            (long long)ncell, need, (size_t)HWENO_NOALLOC_SCRATCH_BYTES);
    char* p = nullptr;
    rc = scratch_address(&p);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    StateBuf U[3];
    for (int k = 0; k < 3; ++k) {
        U[k].u = p; p += ub;
        U[k].d = p; p += db;
    }
    void* H = p; p += db;
    ProbDev* probs = (ProbDev*)p; p += up256(sizeof(ProbDev));
    StepCtl* ctl = (StepCtl*)p; p += up256(sizeof(StepCtl));
    void* tiles = p; p += tb;
    Chunk* chunks = (Chunk*)p;

    // Every value a launch reads is written here first: the table entry and
    // step control come from the arguments (speeds zero, no error, the
    // caller's time), the stage states from state_in.
    ProbDev pd = probdev_of(pr, *cfg, 0, 0);
    pd.t = t;
    pd.dt_in = dt_in;
    StepCtl sc{};
    sc.cfl = cfg->cfl;
    sc.nprob = 1;
    sc.dim = dim;
    const int use_dt_in = dt_in > 0.0;
    const Scheme sch = scheme_of(pr, *cfg);
    const int sgrid = std::max(1, std::min(1024, (std::max(ntiles, nchunks) + 255) / 256));
    noalloc_setup_kernel<<<sgrid, 256, 0, s>>>(pd, sc, probs, ctl, dim, rows, tiles, ntiles,
                                               chunks, nchunks);
    NA_TRY(hipGetLastError());
    NA_TRY(launch_pack(prec, 1, const_cast<double*>(state_in), U[0], 0, 0, K, nvar, ncell, s));
    NA_TRY(launch_alpha(prec, flux, dim, U[0].u, probs, chunks, nchunks, sch, SEL_STALE, 0, s));
    NA_TRY(launch_dt(probs, ctl, 1, use_dt_in, 1, s));
    for (int mode = MODE_S1; mode <= MODE_S3; ++mode) {
        if (mode != MODE_S1 && cfg->alpha_stage) {
            NA_TRY(launch_reset(probs, ctl, 1, SEL_ACTIVE, s));
            NA_TRY(launch_alpha(prec, flux, dim, U[mode - 1].u, probs, chunks, nchunks, sch,
                                SEL_ACTIVE, 0, s));
        }
        StageArgs a{};
        const int k = mode - 1;
        a.in = U[k];
        a.out = U[mode == MODE_S3 ? 0 : k + 1];
        a.un = U[0].u;
        a.h = H;
        a.probs = probs;
        a.tiles = tiles;
        a.ntiles = ntiles;
        a.tile_offset = 0;
        a.sch = sch;
        if (dim == 1) NA_TRY(launch_stage1d(prec, flux, mode, a, 0, s));
        else NA_TRY(launch_stage2d(prec, flux, cfg->gauss_q, mode, 0, a, 0, s));
    }
    NA_TRY(launch_finish(probs, ctl, 1, s));
    NA_TRY(launch_pack(prec, 0, state_out, U[0], 0, 0, K, nvar, ncell, s));
    if (dt_out || bad_out) {
        noalloc_report_kernel<<<1, 64, 0, s>>>(probs, dt_out, bad_out);
        NA_TRY(hipGetLastError());
    }
    return HWENO_OK;
}
