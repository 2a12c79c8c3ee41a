// api.hip -- the C ABI of libturret (declared in include/turret.h): argument
// checks, the device memory plan over caller buffers, the Table 1 call
// sequence with its state checks, HIP graph capture, host copies and
// checkpoints.  All arithmetic of the time step runs in stream_collide.hip,
// kernels.hip and mlp.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/turret.h"
#include "internal.hpp"
#include "lattice.hpp"
#include "mlp.hpp"

using namespace turret;

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int elem_bytes(int storage) { return (storage == LBM_F32 || storage == LBM_MOM) ? 4 : 2; }

struct Plan {
    std::vector<CaseDev> cd;
    std::vector<Tile> tiles;
    std::vector<int> morder;          // internal marker slot -> index in the caller's marker array
    std::vector<MarkerTile> mtiles;
    long long max_tiles = 0;    // tile table capacity: the count at the smallest block (64)
    int Mtot = 0, maxL3 = 0, max_slab = 0;
    int force_surface = 0;    // some case evaluates its force on the parallel surface
    int q = 27;               // populations per cell: 27, or 19 for the D3Q19 comparison lattice
    int planes = 27;          // stored planes per case: q, or 10 with moment storage
    long long pop_elems = 0, reg_cells = 0;
    size_t off_cases, off_body, off_tiles, off_counter, off_mcase, off_xb, off_nb, off_dS, off_X, off_N, off_U, off_hk,
        off_dh, off_part, off_res, off_reg, off_H, off_feat, off_h0, off_hk2, off_hs, off_dSo, off_mtiles, off_tbox, off_log,
        off_mark, off_wt, off_dsh, off_rpop, off_fine0, off_fine1, aux_bytes;
    long long xreg_cells = 0;   // moment storage: cells of all expanded regions (edge L + 2)
    long long fine_elems = 0;   // FP16/BF16 storage: floats of all full-precision boxes (per buffer)
    long long max_box = 0;      // cells of the largest box
    int block = 256;
};

std::string check_case(const lbm_case &c, const lbm_body *b)
{
    char msg[256];
    if (c.nx < 8 || c.ny < 8 || c.nz < 8) return "every dimension must be >= 8";
    if ((long long)c.nx * c.ny * c.nz >= (1LL << 31)) return "a case must have fewer than 2^31 cells";
    if (!(c.tau > 0.5)) return "tau must be > 0.5";
    if (c.sponge_cells < 0 || c.sponge_cells == 1 || c.sponge_cells > c.nz) return "sponge_cells must be 0 or 2..nz";
    for (int bc : {c.bc_zlo, c.bc_zhi})
        if (bc < LBM_BC_PERIODIC || bc > LBM_BC_PRESSURE) return "unknown z boundary code";
    if ((c.bc_zlo == LBM_BC_PERIODIC) != (c.bc_zhi == LBM_BC_PERIODIC)) return "periodic z needs both walls periodic";
    if (c.h_end > 0.0 && std::lround(c.h_ini - c.h_end) >= c.nz) return "window shift exceeds the box height";
    for (int w = 0; w < 2; w++) {
        if (!(std::fabs(c.u_wall[w]) <= 0.2)) return "u_wall must be finite with |u_wall| <= 0.2";
        if (c.u_wall[w] != 0.0 && (w == 0 ? c.bc_zlo : c.bc_zhi) != LBM_BC_NOSLIP)
            return "a moving wall (u_wall != 0) must be a no-slip wall";
    }
    if (b && b->n_markers > 0) {
        if (!b->x_body || !b->n_body || !b->dS) return "marker arrays must not be NULL";
        if (!(b->kappa > 0) || !(b->volume > 0)) return "kappa and volume must be > 0";
        double rb = 0;
        for (int k = 0; k < b->n_markers; k++) {
            double s = 0;
            for (int a = 0; a < 3; a++) s += b->x_body[3 * k + a] * b->x_body[3 * k + a];
            rb = std::max(rb, std::sqrt(s));
        }
        if (!(b->force_offset >= 0.0) || b->force_offset > 64.0) return "force_offset must be in [0, 64]";
        for (int a = 0; a < 3; a++)
            if (!std::isfinite(b->torque[a])) return "external torque must be finite";
        if (b->force_offset > 0.0 && !b->dS_offset) return "force_offset > 0 needs dS_offset";
        const double ro = rb + b->force_offset;   // reach of the force-evaluation points
        const double lo = b->r0[2] - ro, hi = b->r0[2] + ro;
        if (std::floor(lo) - 1 < 0 || std::floor(hi) + 2 > c.nz - 1) {
            std::snprintf(msg, sizeof msg,
                          "markers (or force points) closer than two cells to a z wall (z in [%g, %g], nz %d)", lo, hi,
                          c.nz);
            return msg;
        }
        const int L = (int)std::ceil(2.0 * (1.001 * ro + 0.01)) + 6;
        if (L > c.nx || L > c.ny) return "particle region wider than the box";
        double det = b->J_over_m[0] * (b->J_over_m[4] * b->J_over_m[8] - b->J_over_m[5] * b->J_over_m[7]) -
                     b->J_over_m[1] * (b->J_over_m[3] * b->J_over_m[8] - b->J_over_m[5] * b->J_over_m[6]) +
                     b->J_over_m[2] * (b->J_over_m[3] * b->J_over_m[7] - b->J_over_m[4] * b->J_over_m[6]);
        if (!(std::fabs(det) > 0)) return "J_over_m is singular";
    }
    return "";
}

std::string check_options(const lbm_options *o)
{
    if (!o) return "";
    if (o->storage < LBM_F32 || o->storage > LBM_MOM) return "unknown storage";
    if (o->ibm_cycles < 0 || o->ibm_cycles > 16) return "ibm_cycles must be 1..16 (0 = default 4)";
    if (o->block && o->block != 64 && o->block != 128 && o->block != 256) return "block must be 64, 128 or 256";
    if (o->schedule < 0 || o->schedule > 4) return "schedule must be 0..4";
    if (o->persist_wgs < 0 || o->persist_wgs > (1 << 20)) return "persist_wgs must be 0..2^20";
    if (o->tile_order < 0 || o->tile_order > 2) return "tile_order must be 0, 1 or 2";
    if (o->ibm_diag < 0 || o->ibm_diag > 1) return "ibm_diag must be 0 or 1";
    if (o->forcing < 0 || o->forcing > 1) return "forcing must be 0 or 1";
    if (o->serial_ibm < 0 || o->serial_ibm > 1) return "serial_ibm must be 0 or 1";
    if (o->collision < 0 || o->collision > 1) return "collision must be 0 or 1";
    if (o->lattice != 0 && o->lattice != 19 && o->lattice != 27) return "lattice must be 27 (or 0) or 19";
    if (o->fine_box < 0 || o->fine_box > 1) return "fine_box must be 0 or 1";
    if (o->fine_box && o->storage != LBM_F16 && o->storage != LBM_BF16)
        return "fine_box applies to FP16 and BF16 storage only";
    return "";
}

// Tile table of the lattice kernel: tiles of `block` consecutive cells, in
// case order (0), interleaved round-robin over the cases (1), or with the
// largest cases first (2).
void build_tiles(Plan &P, int block, int order)
{
    const int n = (int)P.cd.size();
    std::vector<int> nt(n), ord(n);
    for (int c = 0; c < n; c++) {
        nt[c] = (int)((P.cd[c].cells + block - 1) / block);
        ord[c] = c;
    }
    if (order == 2)
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return P.cd[a].cells > P.cd[b].cells; });
    auto tile = [&](int c, int t) { return Tile{c, t * block}; };
    P.tiles.clear();
    if (order == 1) {
        const int most = *std::max_element(nt.begin(), nt.end());
        for (int t = 0; t < most; t++)
            for (int c = 0; c < n; c++)
                if (t < nt[c]) P.tiles.push_back(tile(c, t));
    } else {
        for (int c : ord)
            for (int t = 0; t < nt[c]; t++) P.tiles.push_back(tile(c, t));
    }
}

// Tile table of the moment-storage step: one entry per column tile and z
// chunk of each case, `first` holding the tile's index inside its case.
void build_moment_tiles(Plan &P)
{
    P.tiles.clear();
    for (int c = 0; c < (int)P.cd.size(); c++) {
        const int nt = moment_tiles(P.cd[c].nx, P.cd[c].ny, P.cd[c].nz);
        for (int t = 0; t < nt; t++) P.tiles.push_back(Tile{c, t});
    }
}

// Marker order and tiles of one case: sort the markers along a Morton curve
// of their body-frame positions (1.5-cell quantization), then cut the
// sequence into tiles of at most kTileMarkers markers spanning at most
// kTileSpan cells per axis.  The body is rigid, so markers close in the body
// frame stay close in the lab frame.
void tile_markers(const lbm_body &b, int c, int off, std::vector<int> &order, std::vector<MarkerTile> &tiles)
{
    const int M = b.n_markers;
    double lo[3] = {1e300, 1e300, 1e300};
    for (int q = 0; q < M; q++)
        for (int a = 0; a < 3; a++) lo[a] = std::min(lo[a], b.x_body[3 * q + a]);
    std::vector<std::pair<uint64_t, int>> key(M);
    for (int q = 0; q < M; q++) {
        uint64_t k = 0;
        uint32_t cq[3];
        for (int a = 0; a < 3; a++) cq[a] = (uint32_t)std::min(1023.0, (b.x_body[3 * q + a] - lo[a]) / 1.5);
        for (int bit = 9; bit >= 0; bit--)
            for (int a = 0; a < 3; a++) k = (k << 1) | ((cq[a] >> bit) & 1u);
        key[q] = {k, q};
    }
    std::stable_sort(key.begin(), key.end());
    int start = 0;
    double bmin[3], bmax[3];
    for (int j = 0; j < M; j++) {
        const int q = key[j].second;
        bool cut = j - start >= kTileMarkers;
        if (!cut && j > start)
            for (int a = 0; a < 3; a++) {
                const double v = b.x_body[3 * q + a];
                if (std::max(bmax[a], v) - std::min(bmin[a], v) > kTileSpan) cut = true;
            }
        if (cut) {
            tiles.push_back(MarkerTile{c, off + start, j - start, 0});
            start = j;
        }
        if (j == start)
            for (int a = 0; a < 3; a++) bmin[a] = bmax[a] = b.x_body[3 * q + a];
        for (int a = 0; a < 3; a++) {
            bmin[a] = std::min(bmin[a], b.x_body[3 * q + a]);
            bmax[a] = std::max(bmax[a], b.x_body[3 * q + a]);
        }
        order.push_back(q);
    }
    if (M > start) tiles.push_back(MarkerTile{c, off + start, M - start, 0});
}

std::string make_plan(const lbm_case *cases, const lbm_body *bodies, int n, const lbm_options *opt, Plan &P)
{
    if (n < 1 || !cases) return "need at least one case";
    std::string e = check_options(opt);
    if (!e.empty()) return e;
    P.block = (opt && opt->block) ? opt->block : 256;
    const int eb = elem_bytes(opt ? opt->storage : LBM_F32);
    P.q = (opt && opt->lattice == 19) ? 19 : 27;
    if (P.q == 19) {
        if (opt->storage != LBM_F32) return "the D3Q19 lattice runs with FP32 storage";
        if (opt->schedule != 0) return "the D3Q19 lattice runs with schedule 0";
    }
    const bool mom = opt && opt->storage == LBM_MOM;
    if (mom) {
        if (P.q != 27) return "moment storage is a D3Q27 form";
        if (opt->collision != 0) return "moment storage holds regularized states only (collision 0)";
        if (opt->schedule != 0) return "moment storage runs with schedule 0";
    }
    P.planes = mom ? 10 : P.q;
    P.cd.assign(n, CaseDev{});
    long long pop = 0, reg = 0;
    int moff = 0;
    for (int c = 0; c < n; c++) {
        const lbm_case &k = cases[c];
        const lbm_body *b = bodies ? &bodies[c] : nullptr;
        e = check_case(k, b);
        if (!e.empty()) return "case " + std::to_string(c) + ": " + e;
        if (P.q == 19) {
            if (b && b->n_markers > 0) return "case " + std::to_string(c) + ": the D3Q19 lattice is fluid-only (no markers)";
            if (k.bc_zlo != LBM_BC_PERIODIC || k.bc_zhi != LBM_BC_PERIODIC || k.sponge_cells != 0)
                return "case " + std::to_string(c) + ": the D3Q19 lattice needs periodic z and no sponge";
        }
        CaseDev &d = P.cd[c];
        d.nx = k.nx;
        d.ny = k.ny;
        d.nz = k.nz;
        d.bc_lo = k.bc_zlo;
        d.bc_hi = k.bc_zhi;
        d.sponge = k.sponge_cells;
        d.tau0 = (float)k.tau;
        d.forcing = opt ? opt->forcing : 0;
        d.h_ini = k.h_ini;
        d.h_end = k.h_end;
        d.dz = k.h_end > 0.0 ? (int)std::lround(k.h_ini - k.h_end) : 0;
        if (d.dz < 0) d.dz = 0;
        d.cells = (long long)k.nx * k.ny * k.nz;
        // 256-byte aligned direction planes, 1 KB apart from a multiple of
        // 256 bytes: with the planes of a case starting at staggered offsets
        // the lattice kernel's 27-plane pull ran 1.4 % faster at 256 x 256 x 768
        // (where the unpadded stride is a multiple of 64 MiB), in FP32 with
        // 256 elements of pad and in FP16 with 512; other pads from 128 to 768
        // elements were slower
        d.plane = (d.cells + 127) / 128 * 128 + 1024 / eb;
        d.pop_off = pop;
        pop += P.planes * d.plane;
        d.M = b ? std::max(0, b->n_markers) : 0;
        d.force_offset = (b && d.M > 0) ? b->force_offset : 0.0;
        d.uw_lo = (float)k.u_wall[0];
        d.uw_hi = (float)k.u_wall[1];
        if (d.force_offset > 0.0) P.force_surface = 1;
        d.marker_off = moff;
        d.tile_off = (int)P.mtiles.size();
        if (d.M > 0) tile_markers(*b, c, moff, P.morder, P.mtiles);
        d.n_tiles = (int)P.mtiles.size() - d.tile_off;
        moff += d.M;
        if (d.M > 0) {
            double rb = 0;
            for (int q = 0; q < d.M; q++) {
                double s = 0;
                for (int a = 0; a < 3; a++) s += b->x_body[3 * q + a] * b->x_body[3 * q + a];
                rb = std::max(rb, std::sqrt(s));
            }
            d.L = (int)std::ceil(2.0 * (1.001 * (rb + d.force_offset) + 0.01)) + 6;
        } else {
            d.L = 0;
        }
        d.reg_off = reg;
        reg += (long long)d.L * d.L * d.L;
        d.xreg_off = P.xreg_cells;
        if (d.M > 0) P.xreg_cells += (long long)(d.L + 2) * (d.L + 2) * (d.L + 2);
        // full-precision box: the region and a one-cell rim, at most the box
        if (opt && opt->fine_box && d.M > 0) {
            d.LB[0] = std::min(d.L + 2, d.nx);
            d.LB[1] = std::min(d.L + 2, d.ny);
            d.LB[2] = std::min(d.L + 2, d.nz);
            const long long cells = (long long)d.LB[0] * d.LB[1] * d.LB[2];
            d.fine_off = P.fine_elems;
            P.fine_elems += Q * ((cells + 63) / 64 * 64);
            P.max_box = std::max(P.max_box, cells);
        }
        P.maxL3 = std::max(P.maxL3, d.L * d.L * d.L);
        if (d.M > 0) P.max_slab = std::max(P.max_slab, d.dz * k.nx * k.ny);
        P.max_tiles += (d.cells + 63) / 64;
    }
    if (mom)
        build_moment_tiles(P);
    else
        build_tiles(P, P.block, opt ? opt->tile_order : 0);
    P.pop_elems = pop;
    P.reg_cells = reg;
    P.Mtot = moff;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t M = (size_t)std::max(P.Mtot, 1);
    P.off_cases = take(sizeof(CaseDev) * n);
    P.off_body = take(sizeof(BodyDev) * n);
    P.off_tiles = take(sizeof(Tile) * P.max_tiles);
    P.off_counter = take(8 * sizeof(int));
    P.off_mcase = take(sizeof(int) * M);
    P.off_xb = take(sizeof(double) * 3 * M);
    P.off_nb = take(sizeof(double) * 3 * M);
    P.off_dS = take(sizeof(double) * M);
    P.off_X = take(sizeof(double) * 3 * M);
    P.off_N = take(sizeof(double) * 3 * M);
    P.off_U = take(sizeof(double) * 3 * M);
    P.off_hk = take(sizeof(double) * 3 * M);
    P.off_dh = take(sizeof(double) * 3 * M);
    const size_t NT = std::max<size_t>(P.mtiles.size(), 1);
    P.off_part = take(sizeof(double) * kPart * NT);
    P.off_res = take(sizeof(double) * NT);
    P.off_reg = take(sizeof(float) * kRegFields * std::max<long long>(reg, 1));
    P.off_H = take(sizeof(long long) * 3 * kHBufs * std::max<long long>(reg, 1));
    P.off_mark = take((size_t)std::max<long long>(reg, 1));
    P.off_feat = take(sizeof(float) * kMlpIn * M);
    P.off_h0 = take(sizeof(double) * 3 * M);
    P.off_hk2 = take(sizeof(double) * 3 * M);
    P.off_hs = take(sizeof(double) * M);
    P.off_dSo = take(sizeof(double) * M);
    P.off_wt = take(sizeof(double) * 12 * M);
    P.off_dsh = take(sizeof(float) * 4 * std::max<long long>(reg, 1));
    P.off_rpop = take(sizeof(float) * Q * std::max<long long>(mom ? P.xreg_cells : 0, 1));
    P.off_fine0 = take(sizeof(float) * std::max<long long>(P.fine_elems, 1));
    P.off_fine1 = take(sizeof(float) * std::max<long long>(P.fine_elems, 1));
    P.off_mtiles = take(sizeof(MarkerTile) * NT);
    P.off_tbox = take(sizeof(TileBox) * 2 * NT);   // the markers' and the force-surface points' boxes
    P.off_log = take(sizeof(double) * kLogFields * kLogCap * P.cd.size());
    P.aux_bytes = o;
    (void)eb;
    return "";
}

}  // namespace

struct lbm_ctx {
    int n = 0;
    lbm_options opt{};
    hipStream_t stream = nullptr;
    Plan plan;
    std::vector<lbm_case> cases;
    void *pop[2] = {nullptr, nullptr};
    int cur = 0;                  // index of the buffer holding the latest post-collision state
    char *aux = nullptr;
    DevPtrs p{};
    bool has_body = false;
    bool needs_ibm = false;       // lbm_step ran, ibm_couple not yet
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
    int warm_mode = LBM_WARM_NONE;        // start of the multi-direct forcing
    const _Float16 *mlp_th16 = nullptr;   // warm-start network (FP16 weights)
    int mlp_cycles = 0;
    // The coupling of a step reads only the body state and the buffer the
    // lattice kernel reads, so it runs on `side` beside the lattice kernel:
    // `fork` is recorded on `stream` just before the lattice kernel, `join`
    // on `side` after the forcing cycles; the forced correction and
    // everything after it wait for `join` on `stream`.
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::vector<uint32_t> log_read;   // per case: step-log records read so far (the device counts modulo 2^32)
    std::string err;
    ~lbm_ctx()
    {
        if (join) (void)hipEventDestroy(join);
        if (fork) (void)hipEventDestroy(fork);
        if (side) (void)hipStreamDestroy(side);
    }
};

struct lbm_mlp {
    hipStream_t stream = nullptr;
    int max_batch = 0;
    int step = 0;
    float *th32 = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    _Float16 *th16 = nullptr;
    MlpScratch sc{};
    std::string err;
};

static int32_t fail(lbm_ctx *ctx, int32_t code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

static int32_t hip_fail(lbm_ctx *ctx, hipError_t e, const char *where)
{
    return fail(ctx, LBM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr, where)                       \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

// ------------------------------------------ population read without allocation
// lbm_get_populations_noalloc keeps its staging in `scratch`, a file-scope
// device array of kNoAllocScratchBytes that every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name to
// a kernel or a copy: it takes the array's device address once per device
// with hipGetSymbolAddress and uses that address.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch (looked up on its first use).
static int32_t scratch_address(lbm_ctx *ctx, float **out)
{
    int dev = -1;
    HIPCHK(ctx, hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(ctx, LBM_EHIP, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(ctx, LBM_EHIP, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch_ptr[dev] = (float *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

struct DecodeTable {
    double w[27];    // lattice weight of each direction
    float inv[27];   // 1 / s_i of the reduced-precision codecs
};

// Stored values of case c -> populations f = w_i + g_i in the caller's FP64
// layout [q][nz][ny][nx] (physical z, the ring origin undone), with the
// same FP32 decode arithmetic as the host copy of lbm_get_populations.
template <int ST>
__global__ void __launch_bounds__(256) k_decode_populations(const void *__restrict__ raw, long long plane, int q,
                                                            int nx, int ny, int nz, const BodyDev *__restrict__ body,
                                                            DecodeTable tab, double *__restrict__ out)
{
    const long long slab = (long long)nx * ny;
    const long long n = (long long)q * nz * slab;
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int i = (int)(idx / (nz * slab));
    const long long rem = idx - (long long)i * nz * slab;
    const int z = (int)(rem / slab);
    const long long k = rem - (long long)z * slab;
    const int zc = (z + body->z0) % nz;
    const long long src = (long long)i * plane + (long long)zc * slab + k;
    float g;
    if constexpr (ST == LBM_F16) {
        g = (float)((const _Float16 *)raw)[src] * tab.inv[i];
    } else if constexpr (ST == LBM_BF16) {
        g = __uint_as_float((uint32_t)((const uint16_t *)raw)[src] << 16) * tab.inv[i];
    } else {
        g = ((const float *)raw)[src];
    }
    out[idx] = tab.w[i] + (double)g;
}

// The cells of case c's full-precision box of buffer `cur` (when valid):
// f = w_i + g in the caller's layout, over the values k_decode_populations
// wrote from the store.
__global__ void __launch_bounds__(256) k_decode_fine(DevPtrs p, int c, int cur, DecodeTable tab, double *__restrict__ out)
{
    const CaseDev cd = p.cases[c];
    const BodyDev &B = p.body[c];
    if (cd.LB[0] == 0 || !B.fvalid[cur]) return;
    const long long fplane = (long long)cd.LB[0] * cd.LB[1] * cd.LB[2];
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= Q * fplane) return;
    const int i = (int)(idx / fplane);
    const long long slot = idx - (long long)i * fplane;
    const int kx = (int)(slot % cd.LB[0]), ky = (int)((slot / cd.LB[0]) % cd.LB[1]), kz = (int)(slot / (cd.LB[0] * cd.LB[1]));
    const int z = B.fo[cur][2] + kz;
    if (z < 0 || z >= cd.nz) return;
    const int x = ((B.fo[cur][0] + kx) % cd.nx + cd.nx) % cd.nx, y = ((B.fo[cur][1] + ky) % cd.ny + cd.ny) % cd.ny;
    const long long slab = (long long)cd.nx * cd.ny;
    out[((long long)i * cd.nz + z) * slab + (long long)y * cd.nx + x] = tab.w[i] + (double)p.fine[cur][cd.fine_off + idx];
}

static thread_local std::string g_init_error;

extern "C" {

int32_t lbm_required_bytes(const lbm_case *cases, const lbm_body *bodies, int32_t n_cases, const lbm_options *opt,
                           int64_t out_bytes[3])
{
    Plan P;
    std::string e = make_plan(cases, bodies, n_cases, opt, P);
    if (!e.empty()) {
        g_init_error = e;
        return LBM_EINVAL;
    }
    const int eb = elem_bytes(opt ? opt->storage : LBM_F32);
    out_bytes[0] = out_bytes[1] = P.pop_elems * eb;
    out_bytes[2] = (int64_t)P.aux_bytes;
    return LBM_OK;
}

int32_t lbm_init(const lbm_case *cases, const lbm_body *bodies, int32_t n_cases, const lbm_options *opt,
                 const lbm_buffers *buf, const int64_t buf_bytes[3], void *hip_stream, lbm_ctx **out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_ctx *ctx = new lbm_ctx();
    auto bail = [&](int32_t code, const std::string &m) {
        g_init_error = m;
        delete ctx;
        return code;
    };
    std::string e = make_plan(cases, bodies, n_cases, opt, ctx->plan);
    if (!e.empty()) return bail(LBM_EINVAL, e);
    if (!buf || !buf->pop_a || !buf->pop_b || !buf->aux || !buf_bytes) return bail(LBM_EINVAL, "NULL buffer");
    ctx->opt = opt ? *opt : lbm_options{};
    if (ctx->opt.ibm_cycles == 0) ctx->opt.ibm_cycles = 4;
    if (ctx->opt.block == 0) ctx->opt.block = 256;
    if (ctx->opt.schedule >= 2 && ctx->opt.persist_wgs == 0) ctx->opt.persist_wgs = 2048;
    const int eb = elem_bytes(ctx->opt.storage);
    const Plan &P = ctx->plan;
    if (buf_bytes[0] < P.pop_elems * eb || buf_bytes[1] < P.pop_elems * eb || buf_bytes[2] < (int64_t)P.aux_bytes)
        return bail(LBM_ENOMEM, "a buffer is smaller than lbm_required_bytes");
    ctx->n = n_cases;
    ctx->log_read.assign(n_cases, 0u);
    ctx->cases.assign(cases, cases + n_cases);
    ctx->stream = (hipStream_t)hip_stream;
    ctx->pop[0] = buf->pop_a;
    ctx->pop[1] = buf->pop_b;
    ctx->aux = (char *)buf->aux;
    char *a = ctx->aux;
    DevPtrs &p = ctx->p;
    p.cases = (CaseDev *)(a + P.off_cases);
    p.body = (BodyDev *)(a + P.off_body);
    p.tiles = (Tile *)(a + P.off_tiles);
    p.counter = (int *)(a + P.off_counter);
    p.mcase = (int *)(a + P.off_mcase);
    p.xb = (double *)(a + P.off_xb);
    p.nb = (double *)(a + P.off_nb);
    p.dS = (double *)(a + P.off_dS);
    p.X = (double *)(a + P.off_X);
    p.N = (double *)(a + P.off_N);
    p.U = (double *)(a + P.off_U);
    p.hk = (double *)(a + P.off_hk);
    p.dh = (double *)(a + P.off_dh);
    p.part = (double *)(a + P.off_part);
    p.res = (double *)(a + P.off_res);
    p.reg = (float *)(a + P.off_reg);
    p.H = (long long *)(a + P.off_H);
    p.hstride = 3 * std::max<long long>(P.reg_cells, 1);
    p.mark = (unsigned char *)(a + P.off_mark);
    p.wt = (double *)(a + P.off_wt);
    p.dsh = (float *)(a + P.off_dsh);
    p.rpop = (float *)(a + P.off_rpop);
    p.xstride = std::max<long long>(P.xreg_cells, 1);
    p.mtiles = (MarkerTile *)(a + P.off_mtiles);
    p.feat = (float *)(a + P.off_feat);
    p.h0 = (double *)(a + P.off_h0);
    p.hk2 = (double *)(a + P.off_hk2);
    p.hs = (double *)(a + P.off_hs);
    p.dSo = (double *)(a + P.off_dSo);
    p.tbox = (TileBox *)(a + P.off_tbox);
    p.log = (double *)(a + P.off_log);
    p.fine[0] = (float *)(a + P.off_fine0);
    p.fine[1] = (float *)(a + P.off_fine1);

    // host images of the descriptors, body states and markers
    std::vector<BodyDev> bd(n_cases);
    std::vector<int> mcase(std::max(P.Mtot, 1));
    std::vector<double> xb(3 * std::max(P.Mtot, 1)), nb(3 * std::max(P.Mtot, 1)), dS(std::max(P.Mtot, 1));
    std::vector<double> dSo(std::max(P.Mtot, 1), 0.0);
    for (int c = 0; c < n_cases; c++) {
        BodyDev &B = bd[c];
        std::memset(&B, 0, sizeof B);
        const CaseDev &d = P.cd[c];
        B.gravity = cases[c].gravity;
        B.gate = 1e-6;
        B.kappa = 1.0;
        B.vol = 1.0;
        B.d[0] = B.d[4] = B.d[8] = 1.0;
        B.Jm_inv[0] = B.Jm_inv[4] = B.Jm_inv[8] = 1.0;
        if (d.M > 0) {
            const lbm_body &b = bodies[c];
            ctx->has_body = true;
            B.kappa = b.kappa;
            B.vol = b.volume;
            std::memcpy(B.r, b.r0, sizeof B.r);
            std::memcpy(B.d, b.d0, sizeof B.d);
            std::memcpy(B.v, b.v0, sizeof B.v);
            std::memcpy(B.w, b.w0, sizeof B.w);
            std::memcpy(B.Text, b.torque, sizeof B.Text);
            const double *J = b.J_over_m;
            const double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
            const double inv = 1.0 / (J[0] * c00 + J[1] * c01 + J[2] * c02);
            const double Ji[9] = {c00 * inv, (J[2] * J[7] - J[1] * J[8]) * inv, (J[1] * J[5] - J[2] * J[4]) * inv,
                                  c01 * inv, (J[0] * J[8] - J[2] * J[6]) * inv, (J[2] * J[3] - J[0] * J[5]) * inv,
                                  c02 * inv, (J[1] * J[6] - J[0] * J[7]) * inv, (J[0] * J[4] - J[1] * J[3]) * inv};
            std::memcpy(B.Jm_inv, Ji, sizeof Ji);
            double rb = 0;
            for (int j = 0; j < d.M; j++) {
                const int g = d.marker_off + j, q = P.morder[g];   // internal slot g holds marker q
                double s = 0;
                for (int k = 0; k < 3; k++) {
                    xb[3 * g + k] = b.x_body[3 * q + k];
                    nb[3 * g + k] = b.n_body[3 * q + k];
                    s += b.x_body[3 * q + k] * b.x_body[3 * q + k];
                }
                dS[g] = b.dS[q];
                if (d.force_offset > 0.0) dSo[g] = b.dS_offset[q];
                mcase[g] = c;
                rb = std::max(rb, std::sqrt(s));
            }
            B.Rb = 1.001 * (rb + d.force_offset) + 0.01;
            for (int k = 0; k < 3; k++) B.org[k] = (int)std::floor(B.r[k] - B.Rb) - 2;
        }
    }
    hipStream_t s = ctx->stream;
    const size_t popb = (size_t)P.pop_elems * eb;
    hipError_t he;
    if ((he = hipMemsetAsync(ctx->pop[0], 0, popb, s)) != hipSuccess ||
        (he = hipMemsetAsync(ctx->pop[1], 0, popb, s)) != hipSuccess ||
        (he = hipMemsetAsync(ctx->aux, 0, P.aux_bytes, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.cases, P.cd.data(), sizeof(CaseDev) * n_cases, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.body, bd.data(), sizeof(BodyDev) * n_cases, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.tiles, P.tiles.data(), sizeof(Tile) * P.tiles.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.mcase, mcase.data(), sizeof(int) * mcase.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.xb, xb.data(), sizeof(double) * xb.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.nb, nb.data(), sizeof(double) * nb.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.dS, dS.data(), sizeof(double) * dS.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (he = hipMemcpyAsync(p.dSo, dSo.data(), sizeof(double) * dSo.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (P.mtiles.size() &&
         (he = hipMemcpyAsync(p.mtiles, P.mtiles.data(), sizeof(MarkerTile) * P.mtiles.size(), hipMemcpyHostToDevice,
                              s)) != hipSuccess) ||
        (he = hipStreamSynchronize(s)) != hipSuccess)
        return bail(LBM_EHIP, std::string("init: ") + hipGetErrorString(he));
    // side stream of the coupling (default priority, no implicit
    // synchronization with the null stream) and its two events
    if (ctx->has_body &&
        ((he = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking)) != hipSuccess ||
         (he = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming)) != hipSuccess ||
         (he = hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming)) != hipSuccess))
        return bail(LBM_EHIP, std::string("init: side stream: ") + hipGetErrorString(he));
    *out = ctx;
    return LBM_OK;
}

// ------------------------------------------------------------- step calls
static int32_t do_body_advance(lbm_ctx *ctx)
{
    if (!ctx->has_body) return LBM_OK;
    HIPCHK(ctx, launch_body_advance(ctx->p, ctx->n, ctx->stream), "body_advance");
    return LBM_OK;
}

static int32_t do_lbm_step(lbm_ctx *ctx)
{
    const int src = ctx->cur, dst = 1 - ctx->cur;
    if (ctx->has_body) HIPCHK(ctx, hipEventRecord(ctx->fork, ctx->stream), "record fork event");
    if (ctx->opt.storage == LBM_MOM)
        HIPCHK(ctx, launch_moment_step(ctx->pop[src], ctx->pop[dst], ctx->p, (int)ctx->plan.tiles.size(), ctx->stream),
               "lbm_step");
    else if (ctx->plan.q == 19)
        HIPCHK(ctx,
               launch_stream_collide19(ctx->pop[src], ctx->pop[dst], ctx->p, (int)ctx->plan.tiles.size(),
                                       ctx->opt.block, ctx->opt.collision, ctx->stream),
               "lbm_step");
    else
        HIPCHK(ctx,
               launch_stream_collide(ctx->opt.storage, ctx->pop[src], ctx->pop[dst], ctx->p,
                                     (int)ctx->plan.tiles.size(), ctx->opt.block, ctx->opt.schedule,
                                     ctx->opt.persist_wgs, ctx->opt.collision, ctx->stream),
               "lbm_step");
    if (ctx->plan.max_box > 0) {
        // the lattice kernel leaves the box cells to this step, which reads
        // only the buffer the lattice kernel reads: with the coupling beside
        // the lattice kernel it runs on the coupling's stream too, ahead of
        // the coupling (joined before the forced correction)
        const bool beside = ctx->has_body && !ctx->opt.serial_ibm;
        if (beside) HIPCHK(ctx, hipStreamWaitEvent(ctx->side, ctx->fork, 0), "side stream waits for the fork event");
        HIPCHK(ctx,
               launch_fine_step(ctx->opt.storage, ctx->pop[src], ctx->pop[dst], ctx->p, src, dst, ctx->n,
                                ctx->plan.max_box, ctx->opt.collision, beside ? ctx->side : ctx->stream),
               "full-precision box");
    }
    ctx->cur = dst;
    ctx->needs_ibm = ctx->has_body;
    return LBM_OK;
}

static int32_t do_ibm(lbm_ctx *ctx)
{
    if (!ctx->has_body) return LBM_OK;
    const bool serial = ctx->opt.serial_ibm != 0;
    hipStream_t cs = serial ? ctx->stream : ctx->side;
    if (!serial) HIPCHK(ctx, hipStreamWaitEvent(ctx->side, ctx->fork, 0), "side stream waits for the fork event");
    HIPCHK(ctx,
           launch_ibm(ctx->opt.storage, ctx->pop[1 - ctx->cur], ctx->pop[ctx->cur], ctx->p, ctx->n, ctx->plan.Mtot,
                      (int)ctx->plan.mtiles.size(), ctx->plan.maxL3, ctx->opt.ibm_cycles, ctx->warm_mode, ctx->mlp_th16, ctx->mlp_cycles,
                      ctx->opt.ibm_diag, ctx->plan.force_surface, 1 - ctx->cur, cs),
           "ibm_couple");
    if (!serial) {
        HIPCHK(ctx, hipEventRecord(ctx->join, ctx->side), "record join event");
        HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->join, 0), "stream waits for the coupling");
    }
    const int resid_slot =
        ibm_fused(ctx->warm_mode, ctx->opt.ibm_cycles) && !ctx->opt.ibm_diag ? ctx->opt.ibm_cycles - 1 : -1;
    HIPCHK(ctx, launch_correct(ctx->opt.storage, ctx->pop[ctx->cur], ctx->p, ctx->n, ctx->plan.Mtot, ctx->plan.maxL3,
                               ctx->cur, resid_slot, ctx->stream),
           "forced correction");
    ctx->needs_ibm = false;
    return LBM_OK;
}

// advance set: the next step's body advance rides in the window test's kernel
static int32_t do_window(lbm_ctx *ctx, int advance = 0)
{
    if (!ctx->has_body) return LBM_OK;
    HIPCHK(ctx, launch_window(ctx->opt.storage, ctx->pop[ctx->cur], ctx->p, ctx->n, ctx->plan.max_slab, ctx->cur,
                              advance, ctx->stream),
           "window_shift");
    return LBM_OK;
}

int32_t body_advance(lbm_ctx *ctx)
{
    if (!ctx) return LBM_EINVAL;
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "body_advance between lbm_step and ibm_couple");
    return do_body_advance(ctx);
}

int32_t lbm_step(lbm_ctx *ctx)
{
    if (!ctx) return LBM_EINVAL;
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "lbm_step twice without ibm_couple");
    return do_lbm_step(ctx);
}

int32_t ibm_couple(lbm_ctx *ctx)
{
    if (!ctx) return LBM_EINVAL;
    if (ctx->has_body && !ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "ibm_couple without a preceding lbm_step");
    return do_ibm(ctx);
}

int32_t window_shift(lbm_ctx *ctx)
{
    if (!ctx) return LBM_EINVAL;
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "window_shift between lbm_step and ibm_couple");
    return do_window(ctx);
}

// nsteps whole steps in Table 1 order; between two of them the window test
// of one and the body advance of the next share a kernel.
static int32_t run_steps(lbm_ctx *ctx, int nsteps)
{
    if (nsteps <= 0) return LBM_OK;
    int32_t r = do_body_advance(ctx);
    for (int s = 0; s < nsteps && r == LBM_OK; s++) {
        if ((r = do_lbm_step(ctx)) || (r = do_ibm(ctx))) return r;
        r = do_window(ctx, s + 1 < nsteps);
    }
    return r;
}

int32_t lbm_run(lbm_ctx *ctx, int32_t nsteps)
{
    if (!ctx || nsteps < 0) return LBM_EINVAL;
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "lbm_run between lbm_step and ibm_couple");
    return run_steps(ctx, nsteps);
}

static void drop_graph(lbm_ctx *ctx);

int32_t lbm_set_schedule(lbm_ctx *ctx, const lbm_options *opt)
{
    if (!ctx || !opt) return LBM_EINVAL;
    std::string e = check_options(opt);
    if (!e.empty()) return fail(ctx, LBM_EINVAL, e);
    const int cyc = opt->ibm_cycles ? opt->ibm_cycles : 4;
    if (opt->storage != ctx->opt.storage || cyc != ctx->opt.ibm_cycles || opt->forcing != ctx->opt.forcing ||
        (opt->lattice == 19) != (ctx->plan.q == 19) || opt->fine_box != ctx->opt.fine_box)
        return fail(ctx, LBM_EINVAL, "lbm_set_schedule cannot change storage, ibm_cycles, forcing, lattice or fine_box");
    if (ctx->plan.q == 19 && opt->schedule != 0) return fail(ctx, LBM_EINVAL, "the D3Q19 lattice runs with schedule 0");
    if (ctx->opt.storage == LBM_MOM && (opt->schedule != 0 || opt->collision != 0))
        return fail(ctx, LBM_EINVAL, "moment storage runs with schedule 0 and collision 0");
    if (opt->serial_ibm != ctx->opt.serial_ibm || opt->collision != ctx->opt.collision) drop_graph(ctx);
    ctx->opt.serial_ibm = opt->serial_ibm;
    ctx->opt.collision = opt->collision;
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "lbm_set_schedule between lbm_step and ibm_couple");
    const int block = opt->block ? opt->block : 256;
    if (ctx->opt.storage == LBM_MOM)
        build_moment_tiles(ctx->plan);
    else
        build_tiles(ctx->plan, block, opt->tile_order);
    ctx->plan.block = block;
    HIPCHK(ctx, hipMemcpyAsync(ctx->p.tiles, ctx->plan.tiles.data(), sizeof(Tile) * ctx->plan.tiles.size(),
                               hipMemcpyHostToDevice, ctx->stream), "upload tile table");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    drop_graph(ctx);
    ctx->opt.block = block;
    ctx->opt.schedule = opt->schedule;
    ctx->opt.persist_wgs = opt->schedule >= 2 && opt->persist_wgs == 0 ? 2048 : opt->persist_wgs;
    ctx->opt.tile_order = opt->tile_order;
    return LBM_OK;
}

// ---------------------------------------------------------------- graphs
static void drop_graph(lbm_ctx *ctx)
{
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    ctx->gsteps = 0;
}

int32_t lbm_graph_capture(lbm_ctx *ctx, int32_t steps)
{
    if (!ctx) return LBM_EINVAL;
    if (steps < 2 || steps % 2) return fail(ctx, LBM_EINVAL, "steps_per_graph must be even and >= 2");
    if (!ctx->stream) return fail(ctx, LBM_EINVAL, "graph capture needs a non-default stream");
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "capture between lbm_step and ibm_couple");
    drop_graph(ctx);
    const int cur0 = ctx->cur;
    HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    int32_t r = run_steps(ctx, steps);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    ctx->cur = cur0;
    ctx->needs_ibm = false;
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
    ctx->graph = g;
    e = hipGraphInstantiateWithFlags(&ctx->gexec, g, 0);
    if (e != hipSuccess) {
        drop_graph(ctx);
        return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    ctx->gsteps = steps;
    return LBM_OK;
}

int32_t lbm_graph_launch(lbm_ctx *ctx)
{
    if (!ctx) return LBM_EINVAL;
    if (!ctx->gexec) return fail(ctx, LBM_ESTATE, "no captured graph");
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "graph launch between lbm_step and ibm_couple");
    HIPCHK(ctx, hipGraphLaunch(ctx->gexec, ctx->stream), "hipGraphLaunch");
    return LBM_OK;
}

// ------------------------------------------------------------ host copies
// Weight of direction i: D3Q27, or D3Q19 (the D3Q27 order with the corners
// left out: 1/3, 1/18, 1/36).
static double lattice_weight(int q, int i)
{
    if (q == 27) return wq(i);
    int j = 0;
    for (int k = 0; k < 27; k++) {
        const int n = (k % 3 - 1) * (k % 3 - 1) + ((k / 3) % 3 - 1) * ((k / 3) % 3 - 1) + (k / 9 - 1) * (k / 9 - 1);
        if (n == 3) continue;
        if (j == i) return n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        j++;
    }
    return 0.0;
}

static float host_dec(int storage, const void *raw, size_t idx, int i)
{
    const double inv = 1.0 / store_scale(i);
    if (storage == LBM_F32) return ((const float *)raw)[idx];
    if (storage == LBM_F16) return (float)((const _Float16 *)raw)[idx] * (float)inv;
    uint32_t u = (uint32_t)((const uint16_t *)raw)[idx] << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f * (float)inv;
}

static void host_enc(int storage, void *raw, size_t idx, int i, float g)
{
    const float sc = (float)store_scale(i);
    if (storage == LBM_F32) {
        ((float *)raw)[idx] = g;
    } else if (storage == LBM_F16) {
        ((_Float16 *)raw)[idx] = (_Float16)(g * sc);
    } else {
        float f = g * sc;
        uint32_t u;
        std::memcpy(&u, &f, 4);
        if ((u & 0x7fffffffu) > 0x7f800000u) u = (u >> 16) | 0x40u;
        else u = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
        ((uint16_t *)raw)[idx] = (uint16_t)u;
    }
}

static int32_t read_body(lbm_ctx *ctx, int c, BodyDev &B)
{
    HIPCHK(ctx, hipMemcpyAsync(&B, ctx->p.body + c, sizeof B, hipMemcpyDeviceToHost, ctx->stream), "read body");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    return LBM_OK;
}

int32_t lbm_get_populations(lbm_ctx *ctx, int32_t c, double *out)
{
    if (!ctx || !out || c < 0 || c >= ctx->n) return fail(ctx, LBM_EINVAL, "bad case or NULL output");
    BodyDev B;
    int32_t r = read_body(ctx, c, B);
    if (r) return r;
    const CaseDev &d = ctx->plan.cd[c];
    const bool mom = ctx->opt.storage == LBM_MOM;
    const int st = mom ? LBM_F32 : ctx->opt.storage;
    const int eb = elem_bytes(st);
    const int q = ctx->plan.q;
    std::vector<char> raw((size_t)q * d.plane * eb);
    const char *src = (const char *)ctx->pop[ctx->cur] + (size_t)d.pop_off * eb;
    if (mom) {   // reconstruct the populations on the device
        float *tmp = nullptr;
        HIPCHK(ctx, hipMalloc(&tmp, raw.size()), "allocate population buffer");
        hipError_t he = launch_moments_expand((const float *)src, tmp, ctx->p, c, ctx->stream);
        if (he == hipSuccess) he = hipMemcpyAsync(raw.data(), tmp, raw.size(), hipMemcpyDeviceToHost, ctx->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
        (void)hipFree(tmp);
        HIPCHK(ctx, he, "reconstruct populations");
    } else {
        HIPCHK(ctx, hipMemcpyAsync(raw.data(), src, raw.size(), hipMemcpyDeviceToHost, ctx->stream), "copy populations");
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    }
    const size_t slab = (size_t)d.nx * d.ny;
    for (int i = 0; i < q; i++)
        for (int z = 0; z < d.nz; z++) {
            const int zc = (z + B.z0) % d.nz;
            for (size_t k = 0; k < slab; k++)
                out[((size_t)i * d.nz + z) * slab + k] =
                    lattice_weight(q, i) + (double)host_dec(st, raw.data(), (size_t)i * d.plane + zc * slab + k, i);
        }
    // cells of the full-precision box: their FP32 values
    if (d.LB[0] > 0 && B.fvalid[ctx->cur]) {
        const long long fplane = (long long)d.LB[0] * d.LB[1] * d.LB[2];
        std::vector<float> fb((size_t)Q * fplane);
        HIPCHK(ctx, hipMemcpyAsync(fb.data(), ctx->p.fine[ctx->cur] + d.fine_off, fb.size() * sizeof(float),
                                   hipMemcpyDeviceToHost, ctx->stream), "copy the full-precision box");
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
        const int *fo = B.fo[ctx->cur];
        for (int kz = 0; kz < d.LB[2]; kz++) {
            const int z = fo[2] + kz;
            if (z < 0 || z >= d.nz) continue;
            for (int ky = 0; ky < d.LB[1]; ky++)
                for (int kx = 0; kx < d.LB[0]; kx++) {
                    const int x = ((fo[0] + kx) % d.nx + d.nx) % d.nx, y = ((fo[1] + ky) % d.ny + d.ny) % d.ny;
                    const long long slot = ((long long)kz * d.LB[1] + ky) * d.LB[0] + kx;
                    for (int i = 0; i < Q; i++)
                        out[((size_t)i * d.nz + z) * slab + (size_t)y * d.nx + x] =
                            lattice_weight(q, i) + (double)fb[(size_t)i * fplane + slot];
                }
        }
    }
    return B.err ? fail(ctx, LBM_EUNSTABLE, "unstable: marker stencil left the box or non-finite IBM value") : LBM_OK;
}

int32_t lbm_set_populations(lbm_ctx *ctx, int32_t c, const double *in)
{
    if (!ctx || !in || c < 0 || c >= ctx->n) return fail(ctx, LBM_EINVAL, "bad case or NULL input");
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "set_populations between lbm_step and ibm_couple");
    BodyDev B;
    int32_t r = read_body(ctx, c, B);
    if (r) return r;
    const CaseDev &d = ctx->plan.cd[c];
    const bool mom = ctx->opt.storage == LBM_MOM;
    const int st = mom ? LBM_F32 : ctx->opt.storage;
    const int eb = elem_bytes(st);
    const int q = ctx->plan.q;
    std::vector<char> raw((size_t)q * d.plane * eb);
    const size_t slab = (size_t)d.nx * d.ny;
    for (int i = 0; i < q; i++)
        for (int z = 0; z < d.nz; z++) {
            const int zc = (z + B.z0) % d.nz;
            for (size_t k = 0; k < slab; k++)
                host_enc(st, raw.data(), (size_t)i * d.plane + zc * slab + k, i,
                         (float)(in[((size_t)i * d.nz + z) * slab + k] - lattice_weight(q, i)));
        }
    char *dst = (char *)ctx->pop[ctx->cur] + (size_t)d.pop_off * eb;
    if (mom) {   // project onto the stored moments on the device
        float *tmp = nullptr;
        HIPCHK(ctx, hipMalloc(&tmp, raw.size()), "allocate population buffer");
        hipError_t he = hipMemcpyAsync(tmp, raw.data(), raw.size(), hipMemcpyHostToDevice, ctx->stream);
        if (he == hipSuccess) he = launch_moments_project(tmp, (float *)dst, d.plane, d.cells, ctx->stream);
        // the forcing shifts of the last correction no longer apply
        const int zero = 0;
        if (he == hipSuccess)
            he = hipMemcpyAsync(&ctx->p.body[c].dvalid, &zero, sizeof zero, hipMemcpyHostToDevice, ctx->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
        (void)hipFree(tmp);
        HIPCHK(ctx, he, "project populations");
    } else {
        HIPCHK(ctx, hipMemcpyAsync(dst, raw.data(), raw.size(), hipMemcpyHostToDevice, ctx->stream), "copy populations");
        if (d.LB[0] > 0) {   // the full-precision box restarts from the rounded values
            const int zero = 0;
            HIPCHK(ctx, hipMemcpyAsync(&ctx->p.body[c].fvalid[ctx->cur], &zero, sizeof zero, hipMemcpyHostToDevice,
                                       ctx->stream), "reset the full-precision box");
        }
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    }
    return LBM_OK;
}

int32_t lbm_get_populations_noalloc(lbm_ctx *ctx, int32_t c, double *dev_out)
{
    if (!ctx || !dev_out || c < 0 || c >= ctx->n) return fail(ctx, LBM_EINVAL, "bad case or NULL output");
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "population read between lbm_step and ibm_couple");
    const CaseDev &d = ctx->plan.cd[c];
    const bool mom = ctx->opt.storage == LBM_MOM;
    const int st = mom ? LBM_F32 : ctx->opt.storage;
    const int q = ctx->plan.q;
    const size_t staged = (size_t)q * (size_t)d.plane * sizeof(float);
    if (mom && staged > kNoAllocScratchBytes)
        return fail(ctx, LBM_EINVAL,
                    "case too large for the no-allocation read: moment storage stages " + std::to_string(staged) +
                        " bytes, the scratch holds " + std::to_string(kNoAllocScratchBytes));
    DecodeTable tab{};
    for (int i = 0; i < q; i++) {
        tab.w[i] = lattice_weight(q, i);
        tab.inv[i] = (float)(1.0 / store_scale(i));
    }
    const void *raw = (const char *)ctx->pop[ctx->cur] + (size_t)d.pop_off * elem_bytes(st);
    if (mom) {
        float *sp = nullptr;
        int32_t r = scratch_address(ctx, &sp);
        if (r) return r;
        HIPCHK(ctx, launch_moments_expand_n((const float *)raw, sp, ctx->p, c, d.cells, ctx->stream),
               "reconstruct populations in the scratch");
        raw = sp;
    }
    const long long n = (long long)q * d.cells;
    const dim3 grid((unsigned)((n + 255) / 256));
    const BodyDev *body = ctx->p.body + c;
    switch (st) {
    case LBM_F16:
        hipLaunchKernelGGL(k_decode_populations<LBM_F16>, grid, dim3(256), 0, ctx->stream, raw, d.plane, q, d.nx, d.ny,
                           d.nz, body, tab, dev_out);
        break;
    case LBM_BF16:
        hipLaunchKernelGGL(k_decode_populations<LBM_BF16>, grid, dim3(256), 0, ctx->stream, raw, d.plane, q, d.nx,
                           d.ny, d.nz, body, tab, dev_out);
        break;
    default:
        hipLaunchKernelGGL(k_decode_populations<LBM_F32>, grid, dim3(256), 0, ctx->stream, raw, d.plane, q, d.nx, d.ny,
                           d.nz, body, tab, dev_out);
        break;
    }
    HIPCHK(ctx, hipGetLastError(), "decode populations");
    if (d.LB[0] > 0) {
        const long long nf = (long long)Q * d.LB[0] * d.LB[1] * d.LB[2];
        hipLaunchKernelGGL(k_decode_fine, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, ctx->stream, ctx->p, c,
                           ctx->cur, tab, dev_out);
        HIPCHK(ctx, hipGetLastError(), "decode the full-precision box");
    }
    return LBM_OK;
}

int32_t body_get_state(lbm_ctx *ctx, int32_t c, double out[32])
{
    if (!ctx || !out || c < 0 || c >= ctx->n) return fail(ctx, LBM_EINVAL, "bad case or NULL output");
    BodyDev B;
    int32_t r = read_body(ctx, c, B);
    if (r) return r;
    std::memcpy(out, B.r, 3 * sizeof(double));
    std::memcpy(out + 3, B.d, 9 * sizeof(double));
    std::memcpy(out + 12, B.v, 3 * sizeof(double));
    std::memcpy(out + 15, B.w, 3 * sizeof(double));
    std::memcpy(out + 18, B.F, 3 * sizeof(double));
    std::memcpy(out + 21, B.T, 3 * sizeof(double));
    std::memcpy(out + 24, B.Fp, 3 * sizeof(double));
    out[27] = B.resid;
    out[28] = B.steps;
    out[29] = B.shifts;
    out[30] = B.z0;
    out[31] = B.err;
    return B.err ? fail(ctx, LBM_EUNSTABLE, "unstable: marker stencil left the box or non-finite IBM value") : LBM_OK;
}

// ------------------------------------------------------------ checkpoints
static const char kMagic[8] = {'T', 'U', 'R', 'R', 'E', 'T', '0', '1'};

int32_t lbm_save(lbm_ctx *ctx, const char *path)
{
    if (!ctx || !path) return LBM_EINVAL;
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "save between lbm_step and ibm_couple");
    const int eb = elem_bytes(ctx->opt.storage);
    // moment storage also keeps the forcing shifts of the last correction,
    // FP16/BF16 storage the full-precision boxes of the current buffer
    const size_t extra = ctx->opt.storage == LBM_MOM
                             ? sizeof(float) * 4 * (size_t)std::max<long long>(ctx->plan.reg_cells, 1)
                             : sizeof(float) * (size_t)ctx->plan.fine_elems;
    const void *extra_src = ctx->opt.storage == LBM_MOM ? (const void *)ctx->p.dsh : (const void *)ctx->p.fine[ctx->cur];
    const size_t popb = (size_t)ctx->plan.pop_elems * eb;
    std::vector<char> pop(popb + extra);
    std::vector<BodyDev> bd(ctx->n);
    HIPCHK(ctx, hipMemcpyAsync(pop.data(), ctx->pop[ctx->cur], popb, hipMemcpyDeviceToHost, ctx->stream), "save");
    if (extra)
        HIPCHK(ctx, hipMemcpyAsync(pop.data() + popb, extra_src, extra, hipMemcpyDeviceToHost, ctx->stream), "save");
    HIPCHK(ctx, hipMemcpyAsync(bd.data(), ctx->p.body, sizeof(BodyDev) * ctx->n, hipMemcpyDeviceToHost, ctx->stream), "save");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    for (BodyDev &b : bd) {   // the file keeps the current buffer's box in slot 0
        if (ctx->cur == 1) std::memcpy(b.fo[0], b.fo[1], sizeof b.fo[0]);
        b.fvalid[0] = b.fvalid[ctx->cur];
        b.fvalid[1] = 0;
    }
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(ctx, LBM_EINVAL, std::string("cannot open ") + path);
    const int64_t hdr[4] = {ctx->n, ctx->opt.storage, (int64_t)popb, (int64_t)sizeof(BodyDev)};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              std::fwrite(bd.data(), sizeof(BodyDev), ctx->n, f) == (size_t)ctx->n &&
              std::fwrite(pop.data(), 1, popb + extra, f) == popb + extra;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? LBM_OK : fail(ctx, LBM_EINVAL, "write failed");
}

int32_t lbm_load(lbm_ctx *ctx, const char *path)
{
    if (!ctx || !path) return LBM_EINVAL;
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "load between lbm_step and ibm_couple");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, LBM_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int64_t hdr[4];
    const int eb = elem_bytes(ctx->opt.storage);
    const size_t extra = ctx->opt.storage == LBM_MOM
                             ? sizeof(float) * 4 * (size_t)std::max<long long>(ctx->plan.reg_cells, 1)
                             : sizeof(float) * (size_t)ctx->plan.fine_elems;
    void *extra_dst = ctx->opt.storage == LBM_MOM ? (void *)ctx->p.dsh : (void *)ctx->p.fine[ctx->cur];
    const size_t popb = (size_t)ctx->plan.pop_elems * eb;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == ctx->n && hdr[1] == ctx->opt.storage &&
              hdr[2] == (int64_t)popb && hdr[3] == (int64_t)sizeof(BodyDev);
    std::vector<BodyDev> bd(ctx->n);
    std::vector<char> pop(ok ? popb + extra : 0);
    ok = ok && std::fread(bd.data(), sizeof(BodyDev), ctx->n, f) == (size_t)ctx->n &&
         std::fread(pop.data(), 1, popb + extra, f) == popb + extra;
    std::fclose(f);
    if (!ok) return fail(ctx, LBM_EINVAL, "checkpoint does not match this context");
    for (BodyDev &b : bd) {   // slot 0 of the file is the current buffer's box
        if (ctx->cur == 1) std::memcpy(b.fo[1], b.fo[0], sizeof b.fo[0]);
        b.fvalid[ctx->cur] = b.fvalid[0];
        b.fvalid[1 - ctx->cur] = 0;
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->pop[ctx->cur], pop.data(), popb, hipMemcpyHostToDevice, ctx->stream), "load");
    if (extra)
        HIPCHK(ctx, hipMemcpyAsync(extra_dst, pop.data() + popb, extra, hipMemcpyHostToDevice, ctx->stream), "load");
    HIPCHK(ctx, hipMemcpyAsync(ctx->p.body, bd.data(), sizeof(BodyDev) * ctx->n, hipMemcpyHostToDevice, ctx->stream), "load");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    for (int c = 0; c < ctx->n; c++) ctx->log_read[c] = bd[c].logged;   // the ring holds none of the loaded steps
    return LBM_OK;
}

// ------------------------------------------------------------- step log
int32_t lbm_log_read(lbm_ctx *ctx, int32_t c, double *out, int32_t max_records, int32_t *n_read, int64_t *n_lost)
{
    if (!ctx || c < 0 || c >= ctx->n || max_records < 0 || !n_read || (max_records > 0 && !out))
        return fail(ctx, LBM_EINVAL, "lbm_log_read: bad case, negative count or NULL output");
    *n_read = 0;
    if (n_lost) *n_lost = 0;
    BodyDev B;
    int32_t r = read_body(ctx, c, B);   // synchronizes: every launched step has written its record
    if (r) return r;
    uint32_t &cur = ctx->log_read[c];
    uint32_t avail = B.logged - cur;
    if (avail > (uint32_t)kLogCap) {
        if (n_lost) *n_lost = avail - (uint32_t)kLogCap;
        cur = B.logged - (uint32_t)kLogCap;
        avail = kLogCap;
    }
    const int n = (int)std::min<uint32_t>(avail, (uint32_t)max_records);
    if (n == 0) return LBM_OK;
    const double *ring = ctx->p.log + (size_t)c * kLogCap * kLogFields;
    const int slot = (int)(cur % (uint32_t)kLogCap);
    const int first = std::min(n, kLogCap - slot);
    const size_t rb = sizeof(double) * kLogFields;
    HIPCHK(ctx, hipMemcpyAsync(out, ring + (size_t)slot * kLogFields, rb * first, hipMemcpyDeviceToHost, ctx->stream),
           "read the step log");
    if (n > first)
        HIPCHK(ctx, hipMemcpyAsync(out + (size_t)first * kLogFields, ring, rb * (n - first), hipMemcpyDeviceToHost,
                                   ctx->stream),
               "read the step log");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    cur += (uint32_t)n;
    *n_read = n;
    return LBM_OK;
}

// ------------------------------------------------------- learned warm start
static_assert(LBM_MLP_IN == kMlpIn && LBM_MLP_PARAMS == kMlpParams, "network sizes of the header");

static size_t mlp_layout(int max_batch, size_t off[12])
{
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t P = kMlpParams, n = (size_t)max_batch;
    const size_t slices = (n + kMlpSlice - 1) / kMlpSlice, blocks = (n + 255) / 256;
    off[0] = take(4 * P);                      // th32
    off[1] = take(2 * P);                      // th16
    off[2] = take(4 * P);                      // m
    off[3] = take(4 * P);                      // v
    off[4] = take(4 * P);                      // grad
    off[5] = take(4);                          // loss
    off[6] = take(4 * n * 4 * kMlpH);          // a1 a2 d1 d2
    off[7] = take(4 * n * 2 * kMlpH);          // dz1 dz2
    off[8] = take(4 * n * kMlpOut);            // dy
    off[9] = take(4 * slices * P);             // gradient partials
    off[10] = take(4 * blocks);                // loss partials
    return o;
}

int32_t mlp_required_bytes(int32_t max_batch, int64_t *out_bytes)
{
    if (max_batch < 1 || max_batch > (1 << 20) || !out_bytes) {
        g_init_error = "mlp_required_bytes: max_batch must be 1..2^20";
        return LBM_EINVAL;
    }
    size_t off[12];
    *out_bytes = (int64_t)mlp_layout(max_batch, off);
    return LBM_OK;
}

int32_t mlp_create(void *dev_buf, int64_t bytes, int32_t max_batch, void *hip_stream, lbm_mlp **out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    int64_t need = 0;
    if (mlp_required_bytes(max_batch, &need)) return LBM_EINVAL;
    if (!dev_buf) {
        g_init_error = "mlp_create: NULL buffer";
        return LBM_EINVAL;
    }
    if (bytes < need) {
        g_init_error = "mlp_create: buffer smaller than mlp_required_bytes";
        return LBM_ENOMEM;
    }
    lbm_mlp *m = new lbm_mlp();
    size_t off[12];
    mlp_layout(max_batch, off);
    char *b = (char *)dev_buf;
    m->stream = (hipStream_t)hip_stream;
    m->max_batch = max_batch;
    m->th32 = (float *)(b + off[0]);
    m->th16 = (_Float16 *)(b + off[1]);
    m->m = (float *)(b + off[2]);
    m->v = (float *)(b + off[3]);
    m->grad = (float *)(b + off[4]);
    m->loss = (float *)(b + off[5]);
    const size_t n = (size_t)max_batch;
    float *act = (float *)(b + off[6]);
    m->sc.a1 = act;
    m->sc.a2 = act + n * kMlpH;
    m->sc.d1 = act + 2 * n * kMlpH;
    m->sc.d2 = act + 3 * n * kMlpH;
    float *dz = (float *)(b + off[7]);
    m->sc.dz1 = dz;
    m->sc.dz2 = dz + n * kMlpH;
    m->sc.dy = (float *)(b + off[8]);
    m->sc.part = (float *)(b + off[9]);
    m->sc.loss_part = (float *)(b + off[10]);
    hipError_t e = hipMemsetAsync(dev_buf, 0, (size_t)need, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        g_init_error = std::string("mlp_create: ") + hipGetErrorString(e);
        delete m;
        return LBM_EHIP;
    }
    *out = m;
    return LBM_OK;
}

static int32_t mlp_fail(lbm_mlp *m, int32_t code, const std::string &msg)
{
    if (m) m->err = msg;
    return code;
}

int32_t mlp_set_params(lbm_mlp *m, const float *host_params)
{
    if (!m || !host_params) return LBM_EINVAL;
    hipError_t e = hipMemcpyAsync(m->th32, host_params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, sizeof(float) * kMlpParams, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, sizeof(float) * kMlpParams, m->stream);
    if (e == hipSuccess) e = launch_mlp_round(m->th32, m->th16, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return mlp_fail(m, LBM_EHIP, std::string("mlp_set_params: ") + hipGetErrorString(e));
    m->step = 0;
    return LBM_OK;
}

int32_t mlp_get_params(lbm_mlp *m, float *host_params)
{
    if (!m || !host_params) return LBM_EINVAL;
    hipError_t e = hipMemcpyAsync(host_params, m->th32, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return mlp_fail(m, LBM_EHIP, std::string("mlp_get_params: ") + hipGetErrorString(e));
    return LBM_OK;
}

int32_t mlp_forward(lbm_mlp *m, const float *dev_x, int32_t n, float *dev_y)
{
    if (!m || !dev_x || !dev_y || n < 1) return m ? mlp_fail(m, LBM_EINVAL, "mlp_forward: bad arguments") : LBM_EINVAL;
    hipError_t e = launch_mlp_forward(m->th16, dev_x, n, dev_y, m->stream);
    if (e != hipSuccess) return mlp_fail(m, LBM_EHIP, std::string("mlp_forward: ") + hipGetErrorString(e));
    return LBM_OK;
}

int32_t mlp_grad(lbm_mlp *m, const float *dev_x, const float *dev_t, int32_t n, float *dev_grad, float *dev_loss)
{
    if (!m || !dev_x || !dev_t || n < 1 || n > m->max_batch)
        return m ? mlp_fail(m, LBM_EINVAL, "mlp_grad: bad arguments or n > max_batch") : LBM_EINVAL;
    hipError_t e = launch_mlp_grad(m->th16, dev_x, dev_t, n, m->sc, dev_grad ? dev_grad : m->grad,
                                   dev_loss ? dev_loss : m->loss, m->stream);
    if (e != hipSuccess) return mlp_fail(m, LBM_EHIP, std::string("mlp_grad: ") + hipGetErrorString(e));
    return LBM_OK;
}

int32_t mlp_train_step(lbm_mlp *m, const float *dev_x, const float *dev_t, int32_t n, float lr, float *dev_loss)
{
    int32_t r = mlp_grad(m, dev_x, dev_t, n, nullptr, dev_loss);
    if (r) return r;
    m->step += 1;
    hipError_t e = launch_mlp_adam(m->th32, m->th16, m->m, m->v, m->grad, lr, m->step, m->stream);
    if (e != hipSuccess) return mlp_fail(m, LBM_EHIP, std::string("mlp_train_step: ") + hipGetErrorString(e));
    return LBM_OK;
}

const char *mlp_last_error(const lbm_mlp *m) { return m ? m->err.c_str() : g_init_error.c_str(); }

int32_t mlp_destroy(lbm_mlp *m)
{
    delete m;
    return LBM_OK;
}

int32_t lbm_set_warm_start(lbm_ctx *ctx, int32_t mode, const lbm_mlp *m, int32_t cycles)
{
    if (!ctx) return LBM_EINVAL;
    if (mode < LBM_WARM_NONE || mode > LBM_WARM_MLP) return fail(ctx, LBM_EINVAL, "unknown warm-start mode");
    if (mode == LBM_WARM_MLP && !m) return fail(ctx, LBM_EINVAL, "network warm start needs a network");
    if (mode != LBM_WARM_NONE && (cycles < 1 || cycles > 8)) return fail(ctx, LBM_EINVAL, "cycles must be 1..8");
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "warm-start change between lbm_step and ibm_couple");
    drop_graph(ctx);
    ctx->warm_mode = mode;
    ctx->mlp_th16 = mode == LBM_WARM_MLP ? m->th16 : nullptr;
    ctx->mlp_cycles = mode == LBM_WARM_NONE ? 0 : cycles;
    return LBM_OK;
}

int32_t lbm_set_ibm_gate(lbm_ctx *ctx, int32_t c, double threshold)
{
    if (!ctx || c < 0 || c >= ctx->n || !(threshold >= 0)) return fail(ctx, LBM_EINVAL, "bad case or threshold");
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "set_ibm_gate between lbm_step and ibm_couple");
    HIPCHK(ctx, hipMemcpyAsync(&ctx->p.body[c].gate, &threshold, sizeof(double), hipMemcpyHostToDevice, ctx->stream),
           "set gate");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    return LBM_OK;
}

int32_t lbm_ibm_samples(lbm_ctx *ctx, float *dev_features, float *dev_targets)
{
    if (!ctx || !dev_features || !dev_targets) return fail(ctx, LBM_EINVAL, "NULL output");
    if (ctx->needs_ibm) return fail(ctx, LBM_ESTATE, "samples between lbm_step and ibm_couple");
    const int M = ctx->plan.Mtot;
    if (M == 0) return LBM_OK;
    HIPCHK(ctx, hipMemcpyAsync(dev_features, ctx->p.feat, sizeof(float) * kMlpIn * M, hipMemcpyDeviceToDevice,
                               ctx->stream), "copy features");
    HIPCHK(ctx, launch_targets(ctx->p, M, dev_targets, ctx->stream), "targets");
    return LBM_OK;
}

int32_t lbm_ibm_stats(lbm_ctx *ctx, int32_t c, double out[24])
{
    if (!ctx || !out || c < 0 || c >= ctx->n) return fail(ctx, LBM_EINVAL, "bad case or NULL output");
    BodyDev B;
    int32_t r = read_body(ctx, c, B);
    if (r) return r;
    out[0] = B.resid;
    for (int k = 0; k < 16; k++) out[1 + k] = B.resid_hist[k];
    out[17] = B.accepts;
    out[18] = B.rejects;
    out[19] = B.fallback;
    out[20] = B.warm_cyc_sum;
    out[21] = out[22] = out[23] = 0.0;
    return LBM_OK;
}

int32_t lbm_marker_count(const lbm_ctx *ctx) { return ctx ? ctx->plan.Mtot : -1; }

int64_t lbm_pop_offset(const lbm_ctx *ctx, int32_t c)
{
    if (!ctx || c < 0 || c >= ctx->n) return -1;
    return ctx->plan.cd[c].pop_off;
}

int64_t lbm_plane_stride(const lbm_ctx *ctx, int32_t c)
{
    if (!ctx || c < 0 || c >= ctx->n) return -1;
    return ctx->plan.cd[c].plane;
}

void *lbm_current_buffer(const lbm_ctx *ctx) { return ctx ? ctx->pop[ctx->cur] : nullptr; }

int32_t lbm_stream_copy(void *dst, const void *src, int64_t bytes, void *hip_stream)
{
    if (!dst || !src || bytes <= 0 || bytes % 16) {
        g_init_error = "lbm_stream_copy: NULL pointer or size not a positive multiple of 16";
        return LBM_EINVAL;
    }
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
        g_init_error = std::string("lbm_stream_copy: ") + hipGetErrorString(e);
        return LBM_EHIP;
    }
    return LBM_OK;
}

int32_t lbm_destroy(lbm_ctx *ctx)
{
    if (!ctx) return LBM_OK;
    drop_graph(ctx);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    delete ctx;
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
