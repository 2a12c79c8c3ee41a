// kernels.hip -- gfx950 kernels of the settling-particle time step
// (arXiv 2408.15115, Sec. 2) other than the lattice kernel (stream_collide.hip),
// and their stream launchers.
//
//   k_body_advance        Sec. 2.3: leapfrog / predictor-corrector, FP64
//   k_markers             Sec. 2.3: marker position, normal and rigid velocity;
//                         tile boxes and the marks of the cells they cover
//   k_region_gather       Sec. 2.1 stress and Sec. 2.2 u* on the particle region
//   k_interp_force_tiles  Sec. 2.2: l = 0 interpolation and the stress integral
//                         (+ the first spread); the last tile of a case forms
//                         its FP64 force / torque totals in a fixed order
//   k_spread_tiles        Sec. 2.2 spreading (deterministic fixed-point atomics)
//   k_interp_update_tiles Sec. 2.2 interpolation of u* + H and the residual
//                         (+ the next cycle's spread)
//   k_correct             Sec. 2.2 forced rule: add f0(u + tau h) - f0(u)
//   k_window_*            Sec. 2.5 re-injection as a ring-origin shift
//
// IBM kernels give one 64-lane wavefront to each marker: lane l is the
// stencil node (l & 3, (l >> 2) & 3, l >> 4) of the 4 x 4 x 4 weight support;
// a workgroup takes one tile of nearby markers and stages their common box of
// region cells in LDS.
#include <algorithm>

#include "internal.hpp"
#include "lattice.hpp"
#include "fine.hpp"
#include "pull.hpp"
#include "mlp.hpp"
#include "moments.hpp"
#include <type_traits>

namespace turret {


// ---------------------------------------------------------------- body
__device__ inline void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline void inverse3(const double A[9], double B[9])
{
    const double c00 = A[4] * A[8] - A[5] * A[7];
    const double c01 = A[5] * A[6] - A[3] * A[8];
    const double c02 = A[3] * A[7] - A[4] * A[6];
    const double inv = 1.0 / (A[0] * c00 + A[1] * c01 + A[2] * c02);
    B[0] = c00 * inv;
    B[1] = (A[2] * A[7] - A[1] * A[8]) * inv;
    B[2] = (A[1] * A[5] - A[2] * A[4]) * inv;
    B[3] = c01 * inv;
    B[4] = (A[0] * A[8] - A[2] * A[6]) * inv;
    B[5] = (A[2] * A[3] - A[0] * A[5]) * inv;
    B[6] = c02 * inv;
    B[7] = (A[1] * A[6] - A[0] * A[7]) * inv;
    B[8] = (A[0] * A[4] - A[1] * A[3]) * inv;
}

__device__ inline void mv3(const double A[9], const double x[3], double y[3])
{
#pragma unroll
    for (int a = 0; a < 3; a++) y[a] = A[3 * a] * x[0] + A[3 * a + 1] * x[1] + A[3 * a + 2] * x[2];
}

// Sec. 2.3 leapfrog with F(t), T(t): a = g + F/(kappa V), v(t+1/2), r(t+1);
// w(t+1/2) through M^-1 (J/m)^-1 M with the fluid torque plus the body's
// constant external torque; orientation predictor-corrector.  Then the IBM
// region origin for the new position.
__device__ inline void body_advance_case(const DevPtrs &p, int c)
{
    const CaseDev &cd = p.cases[c];
    BodyDev &B = p.body[c];
    // every field first, in one round of loads (no short-circuit between the
    // two tests, so both loads issue together), then the arithmetic, then the
    // stores
    const int M = cd.M, err = B.err;
    if ((M == 0) | (err != 0)) return;
    const double kappa = B.kappa, vol = B.vol, grav = B.gravity, Rb = B.Rb;
    double F[3], T[3], Te[3], v[3], r[3], w[3], d[9], J[9];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        F[k] = B.F[k];
        T[k] = B.T[k];
        Te[k] = B.Text[k];
        v[k] = B.v[k];
        r[k] = B.r[k];
        w[k] = B.w[k];
    }
#pragma unroll
    for (int k = 0; k < 9; k++) {
        d[k] = B.d[k];
        J[k] = B.Jm_inv[k];
    }
    const int steps = B.steps;
    const double kv = kappa * vol;
    const double a[3] = {F[0] / kv, F[1] / kv, F[2] / kv - grav};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        v[k] += a[k];
        r[k] += v[k];
    }
    double Minv[9], t1[3], t2[3], t3[3];
    inverse3(d, Minv);
    const double Ttot[3] = {T[0] + Te[0], T[1] + Te[1], T[2] + Te[2]};
    mv3(d, Ttot, t1);
    mv3(J, t1, t2);
    mv3(Minv, t2, t3);
#pragma unroll
    for (int k = 0; k < 3; k++) w[k] += t3[k] / kv;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        double di[3] = {d[3 * i], d[3 * i + 1], d[3 * i + 2]}, wd[3], mid[3], wm[3];
        cross3(w, di, wd);
#pragma unroll
        for (int k = 0; k < 3; k++) mid[k] = 0.5 * (di[k] + (di[k] + wd[k]));
        cross3(w, mid, wm);
#pragma unroll
        for (int k = 0; k < 3; k++) d[3 * i + k] = di[k] + wm[k];
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        B.v[k] = v[k];
        B.r[k] = r[k];
        B.w[k] = w[k];
        B.org[k] = (int)floor(r[k] - Rb) - 2;
    }
#pragma unroll
    for (int k = 0; k < 9; k++) B.d[k] = d[k];
    B.steps = steps + 1;
}

__global__ void k_body_advance(DevPtrs p, int n_cases)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n_cases) body_advance_case(p, c);
}

// X_k = r + sum_j xb_kj d_j, n_k = sum_j nb_kj d_j, U_k = v + w x (X_k - r).
// The body fields the region and marker kernels read, copied into registers
// at a kernel's start: after the kernel's first global store the compiler
// must assume the body record may have changed and would reload each field
// with a vector load and a wait of its own.
struct BodyView {
    int err, active;
    int org[3];
    int z0;
    double r[3];
};

__device__ inline BodyView body_view(const BodyDev &B)
{
    BodyView v;
    v.err = B.err;
    v.active = B.active;
    v.z0 = B.z0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        v.org[d] = B.org[d];
        v.r[d] = B.r[d];
    }
    return v;
}

// Moment storage: the tag that selects the moment forms of the region gather,
// the correction and the window reset.
struct CodecMom {
    using T = float;
};

// Moment storage, first pass of the region gather: the collided populations
// (forcing shifts included) of every cell of the particle region and a
// one-cell rim, edge E = L + 2, into rpop.  Rim planes beyond a z wall are
// never pulled and are left alone.
__global__ void k_region_expand_mom(const float *__restrict__ src, DevPtrs p)
{
    const int c = blockIdx.y;
    const CaseDev cd = p.cases[c];
    const BodyView B = body_view(p.body[c]);
    if (cd.M == 0 || B.err != 0) return;
    const int E = cd.L + 2, E3 = E * E * E;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= E3) return;
    const int a = q % E, b = (q / E) % E, cc = q / (E * E);
    int z = B.org[2] - 1 + cc;
    if (z < 0 || z >= cd.nz) {
        if (cd.bc_lo != BC_PERIODIC) return;
        z = wrapi(z, cd.nz);
    }
    const int x = wrapi(B.org[0] - 1 + a, cd.nx), y = wrapi(B.org[1] - 1 + b, cd.ny);
    int slot = z + B.z0;
    if (slot >= cd.nz) slot -= cd.nz;
    const float *sp = src + cd.pop_off + ((long long)slot * cd.ny + y) * cd.nx + x;
    float m[10], sh[4], out[Q];
#pragma unroll
    for (int k = 0; k < 10; k++) m[k] = sp[k * cd.plane];
    (void)mom::shift_at(mom::shift_box(p, cd, p.body[c]), cd.nx, cd.ny, cd.nz, x, y, slot, sh);
    mom::expand(m, sh, out);
    float *dst = p.rpop + cd.xreg_off + q;
#pragma unroll
    for (int i = 0; i < Q; i++) dst[i * p.xstride] = out[i];
}

// Second pass: the pull of pull() from the expanded region, for region cell
// (a, b, cc) at physical height z, with the same z wall rules.
__device__ inline void pull_region(const DevPtrs &p, const CaseDev &cd, int a, int b, int cc, int z, float g[Q])
{
    const int E = cd.L + 2;
    const float *R = p.rpop + cd.xreg_off;
    const int wlo = z == 0 && cd.bc_lo != BC_PERIODIC, whi = z == cd.nz - 1 && cd.bc_hi != BC_PERIODIC;
    Unroll<0, Q>::run([&](auto I) {
        constexpr int i = decltype(I)::value;
        int sa = a + 1 - cx(i), sb = b + 1 - cy(i), sc = cc + 1 - cz(i);
        int dir = i;
        float sign = 1.0f, add = 0.0f;
        if constexpr (cz(i) != 0) {
            const bool wall = cz(i) == 1 ? wlo : whi;
            const int bc = cz(i) == 1 ? cd.bc_lo : cd.bc_hi;
            if (wall) {
                sc = cc + 1;
                if (bc == BC_FREESLIP) {
                    dir = mirror_z(i);
                } else {
                    dir = opposite(i);
                    sa = a + 1;
                    sb = b + 1;
                    if (bc == BC_PRESSURE) sign = -1.0f;
                    else if constexpr (cx(i) != 0) add = (float)(6.0 * wq(i) * cx(i)) * (cz(i) == 1 ? cd.uw_lo : cd.uw_hi);
                }
            }
        }
        g[i] = sign * R[dir * p.xstride + ((long long)sc * E + sb) * E + sa] + add;
    });
}

// ------------------------------------------------------------ region fields
// For every cell of the particle region: pull f(t+1) from the buffer the
// lattice kernel read, then rho - 1, u* = sum xi f / sum f and the stress
// sigma = -p I + (1/(2 tau) - 1) P1 with p = cs^2 (rho - 1) (Sec. 2.1).
// Also clears the fixed-point immersed-force accumulators.  Only cells marked
// by k_markers (inside some tile's stencil box) are visited; the others are
// read by no interpolation and carry no force.
template <class CD>
__global__ void k_region_gather(const typename CD::T *__restrict__ src, DevPtrs p, int sid)
{
    const int c = blockIdx.y;
    const CaseDev cd = p.cases[c];
    const BodyView B = body_view(p.body[c]);
    if (cd.M == 0 || B.err != 0) return;
    const int L = cd.L, L3 = L * L * L;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= L3 || !p.mark[cd.reg_off + q]) return;
    float *R = p.reg + cd.reg_off * kRegFields;
    long long *H = p.H + cd.reg_off * 3;
#pragma unroll
    for (int j = 0; j < kHBufs; j++) {
        H[j * p.hstride + q] = 0;
        H[j * p.hstride + L3 + q] = 0;
        H[j * p.hstride + 2 * L3 + q] = 0;
    }
    const int a = q % L, b = (q / L) % L, cc = q / (L * L);
    const int gz = B.org[2] + cc;
    if (gz < 0 || gz >= cd.nz) {
#pragma unroll
        for (int f = 0; f < kRegFields; f++) R[f * L3 + q] = 0.0f;
        return;
    }
    const int gx = wrapi(B.org[0] + a, cd.nx), gy = wrapi(B.org[1] + b, cd.ny);
    float g[Q];
    if constexpr (std::is_same<CD, CodecMom>::value) {
        pull_region(p, cd, a, b, cc, gz, g);
    } else if (cd.LB[0] > 0) {
        // reduced-precision store with a full-precision box around the body
        const BodyDev &Bd = p.body[c];
        const int fo[3] = {Bd.fo[sid][0], Bd.fo[sid][1], Bd.fo[sid][2]};
        pull_fine<CD>(src + cd.pop_off, Bd.fvalid[sid] ? p.fine[sid] + cd.fine_off : nullptr, cd, B.z0, fo, gx, gy, gz,
                      g);
    } else {
        pull<CD>(src + cd.pop_off, cd.plane, cd.nx, cd.ny, cd.nz, B.z0, cd.bc_lo, cd.bc_hi, cd.uw_lo, cd.uw_hi, gx, gy,
                 gz, g);
    }
    const Macro M = macro(raw_moments(g));
    const float tau = tau_at(cd.tau0, cd.nz, cd.sponge, gz);
    const float fac = 0.5f / tau - 1.0f;
    const float pr = CS2 * M.r1;
    R[0 * L3 + q] = M.r1;
    R[1 * L3 + q] = M.u[0];
    R[2 * L3 + q] = M.u[1];
    R[3 * L3 + q] = M.u[2];
    R[4 * L3 + q] = -pr + fac * M.P[0][0];
    R[5 * L3 + q] = -pr + fac * M.P[1][1];
    R[6 * L3 + q] = -pr + fac * M.P[2][2];
    R[7 * L3 + q] = fac * M.P[0][1];
    R[8 * L3 + q] = fac * M.P[0][2];
    R[9 * L3 + q] = fac * M.P[1][2];
}

// --------------------------------------------------------- marker stencils
// One-dimensional four-point weight function of Sec. 2.2 (two branches).
// Written without branches (one square root per call): the lanes of a
// stencil fall on both branches.
__device__ inline double phi4(double r)
{
    const double a = fabs(r);
    const bool inner = a <= 1.0;
    const double arg = inner ? 1.0 + 4.0 * a - 4.0 * a * a : -7.0 + 12.0 * a - 4.0 * a * a;
    const double sq = sqrt(fmax(arg, 0.0));   // arg >= 1 wherever the value is used
    const double v = inner ? 0.125 * (3.0 - 2.0 * a + sq) : 0.125 * (5.0 - 2.0 * a - sq);
    return a <= 2.0 ? v : 0.0;
}

struct Node {
    int q;        // region cell index, -1 if outside the region
    double W;     // tensor-product weight
};

__device__ inline Node stencil_node(const double X[3], int lane, const CaseDev &cd, const BodyView &B)
{
    const int off[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
    const int n[3] = {cd.nx, cd.ny, cd.nz};
    const int L = cd.L;
    Node nd;
    nd.W = 1.0;
    int r[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int node = (int)floor(X[d]) - 1 + off[d];
        nd.W *= phi4((double)node - X[d]);
        int rel = node - B.org[d];
        if (d < 2) rel = wrapi(rel, n[d]);
        ok = ok && rel >= 0 && rel < L;
        r[d] = rel;
    }
    nd.q = ok ? r[0] + L * (r[1] + L * r[2]) : -1;
    return nd;
}

// v + the value of the lane that the DPP pattern CTRL pairs with this one
// (both 32-bit halves moved by DPP; no LDS traffic).
template <int CTRL>
__device__ inline double dpp_pair_add(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double lane_value(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over a row of 16 lanes (all active), the same bits in every lane of
// the row: pairs (lane ^ 1), quads (lane ^ 2), half rows (mirror of 8) and
// rows (mirror of 16); each step adds the same two operands in both lanes of
// a pair, so the row ends uniform.
__device__ inline double row_sum(double v)
{
    v = dpp_pair_add<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v = dpp_pair_add<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v = dpp_pair_add<0x141>(v);   // row_half_mirror
    v = dpp_pair_add<0x140>(v);   // row_mirror
    return v;
}

// Sum over the 64 lanes of a wavefront (all active), the same bits in every
// lane: row sums, then the four row totals in a fixed order.
__device__ inline double wave_sum(double v)
{
    v = row_sum(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// ------------------------------------------------------------ marker tiles
// One workgroup per marker tile (markers close together on the body): the
// tile's stencils share a box of region cells.  Interpolations stage the
// box's fields in LDS once and read every stencil node from there; spreading
// accumulates into an LDS copy of the box (int64 fixed point) and adds each
// touched cell to HBM once.  A box larger than kBoxCells (not expected for
// the tile span) falls back to per-node HBM access.
// Tile handled by workgroup b: the dispatcher deals workgroups round-robin
// over the 8 XCDs, so consecutive blocks are spread and each XCD is given a
// contiguous (Morton-ordered, hence spatially compact) run of tiles whose
// boxes overlap inside one L2.  The grid is padded to a multiple of 8.
__device__ inline int tile_of_block(int b, int n)
{
    const int per = (n + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

// Box-local index of a lane's stencil node and its weight W = (w_x w_y) w_z
// from the marker's one-dimensional weights w[4 d + o] (k_markers evaluates
// them once per step).
__device__ inline int box_node_w(const double X[3], const double *w, int lane, const TileBox &b, double &W)
{
    const int off[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
    int r[3];
    W = 1.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int node = (int)floor(X[d]) - 1 + off[d];
        W *= w[4 * d + off[d]];
        r[d] = node - b.lo[d];
    }
    return r[0] + b.e[0] * (r[1] + b.e[1] * r[2]);
}

// Lane layout of the interpolation passes: thread t takes marker t / 16 of
// the tile and the stencil column (t & 3, (t >> 2) & 3); its nodes are the
// four z levels of that column.  A row of 16 lanes is one marker, so the
// stencil sums are row sums and the tile's markers run side by side.
static_assert(kTileMarkers * 16 == 256, "one workgroup row of 16 lanes per tile marker");
struct Column {
    int i[4];       // box cells of the four nodes (box path)
    int q[4];       // region cells of the four nodes (per-node path; -1 outside)
    double W[4];    // node weights
};

// The column's nodes from the marker's one-dimensional weights w (box path;
// W = (w_x w_y) w_z, the product order of box_node_w) or from stencil_node.
__device__ inline Column column_nodes(const double X[3], const double *w, int col, const TileBox &tb,
                                      const CaseDev &cd, const BodyView &B)
{
    Column cn;
    const int cx = col & 3, cy = col >> 2;
    if (tb.fits) {
        const double wxy = (1.0 * w[cx]) * w[4 + cy];
        const int b0 = ((int)floor(X[0]) - 1 + cx - tb.lo[0]) +
                       tb.e[0] * (((int)floor(X[1]) - 1 + cy - tb.lo[1]) + tb.e[1] * ((int)floor(X[2]) - 1 - tb.lo[2]));
#pragma unroll
        for (int z = 0; z < 4; z++) {
            cn.W[z] = wxy * w[8 + z];
            cn.i[z] = b0 + z * tb.e[0] * tb.e[1];
            cn.q[z] = -1;
        }
    } else {
#pragma unroll
        for (int z = 0; z < 4; z++) {
            const Node nd = stencil_node(X, col + 16 * z, cd, B);
            cn.W[z] = nd.W;
            cn.q[z] = nd.q;
            cn.i[z] = 0;
        }
    }
    return cn;
}

// Region cell index of box cell i.
__device__ inline int box_region_cell(int i, const TileBox &b, int L)
{
    const int bx = i % b.e[0], t = i / b.e[0], by = t % b.e[1], bz = t / b.e[1];
    return (b.o[0] + bx) + L * ((b.o[1] + by) + L * (b.o[2] + bz));
}

// Marks stencil node `lane` of the point X as used in this step (region
// cells outside every stencil are neither gathered nor corrected).
__device__ inline void mark_node(const DevPtrs &p, const CaseDev &cd, const BodyView &B, const double X[3], int lane)
{
    const int off[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
    const int n[3] = {cd.nx, cd.ny, cd.nz};
    const int L = cd.L;
    int r[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int rel = (int)floor(X[d]) - 1 + off[d] - B.org[d];
        if (d < 2) rel = wrapi(rel, n[d]);
        ok = ok && rel >= 0 && rel < L;
        r[d] = rel;
    }
    if (ok) p.mark[cd.reg_off + r[0] + L * (r[1] + L * r[2])] = 1;
}

// Box of the stencil nodes of the points P held by the lanes with `on` set
// (at least one): first node lo = min floor(P) - 1 and extent
// max floor(P) - min floor(P) + 4 per axis, by butterfly min / max.
__device__ inline void wave_box(const double P[3], bool on, int lo[3], int e[3])
{
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int f = (int)floor(P[d]);
        int mn = on ? f : (1 << 30), mx = on ? f : -(1 << 30);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, __shfl_xor(mn, o));
            mx = max(mx, __shfl_xor(mx, o));
        }
        lo[d] = mn - 1;
        e[d] = mx - mn + 4;
    }
}

// Marks the stencil cells of the tile's points P (lane j < count holds
// point j): the whole box when it lies inside the region, else node by node.
// Returns the box as a TileBox.
__device__ inline TileBox mark_points(const DevPtrs &p, const CaseDev &cd, const BodyView &B, const double P[3],
                                      int count, int lane)
{
    TileBox b;
    wave_box(P, lane < count, b.lo, b.e);
    const int L = cd.L;
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        b.o[d] = b.lo[d] - B.org[d];
        in = in && b.o[d] >= 0 && b.o[d] + b.e[d] <= L;
    }
    const int n = b.e[0] * b.e[1] * b.e[2];
    b.fits = in && n <= kBoxCells;
    if (in) {
        unsigned char *mk = p.mark + cd.reg_off;
        for (int i = lane; i < n; i += 64) mk[box_region_cell(i, b, L)] = 1;
    } else {
        for (int j = 0; j < count; j++) {
            const double Pj[3] = {__shfl(P[0], j), __shfl(P[1], j), __shfl(P[2], j)};
            mark_node(p, cd, B, Pj, lane);
        }
    }
    return b;
}

// One wavefront per marker tile (Sec. 2.3 kinematics): lane j < count forms
// the position, normal and rigid velocity of marker first + j and checks the
// z range; the tile's stencil box goes to the tile table, and the cells of
// that box (and of the force-surface points' box) are marked for this step.
__global__ void __launch_bounds__(64) k_markers(DevPtrs p, int n_mtiles)
{
    const int tix = tile_of_block((int)blockIdx.x, n_mtiles);
    if (tix >= n_mtiles) return;
    const MarkerTile mt = p.mtiles[tix];
    const CaseDev cd = p.cases[mt.c];
    const BodyDev &Bd = p.body[mt.c];
    const BodyView B = body_view(Bd);
    if (B.err != 0) return;
    const int lane = threadIdx.x;
    const bool on = lane < mt.count;
    const int k = mt.first + (on ? lane : 0);
    const double xb[3] = {p.xb[3 * k], p.xb[3 * k + 1], p.xb[3 * k + 2]};
    const double nb[3] = {p.nb[3 * k], p.nb[3 * k + 1], p.nb[3 * k + 2]};
    double X[3], N[3], rel[3], wr[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        X[a] = B.r[a] + xb[0] * Bd.d[a] + xb[1] * Bd.d[3 + a] + xb[2] * Bd.d[6 + a];
        N[a] = nb[0] * Bd.d[a] + nb[1] * Bd.d[3 + a] + nb[2] * Bd.d[6 + a];
        rel[a] = X[a] - B.r[a];
    }
    const double w[3] = {Bd.w[0], Bd.w[1], Bd.w[2]}, vb[3] = {Bd.v[0], Bd.v[1], Bd.v[2]};
    const double dl = cd.force_offset;
    if (on) {
        cross3(w, rel, wr);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            p.X[3 * k + a] = X[a];
            p.N[3 * k + a] = N[a];
            p.U[3 * k + a] = vb[a] + wr[a];
        }
        // the marker's one-dimensional stencil weights for this step
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const int n0 = (int)floor(X[d]) - 1;
#pragma unroll
            for (int o = 0; o < 4; o++) p.wt[12 * k + 4 * d + o] = phi4((double)(n0 + o) - X[d]);
        }
        const int fz = (int)floor(X[2]);
        if (fz - 1 < 0 || fz + 2 > cd.nz - 1) atomicOr(&p.body[mt.c].err, 1);
        if (dl > 0.0) {
            const int gz = (int)floor(X[2] + dl * N[2]);
            if (gz - 1 < 0 || gz + 2 > cd.nz - 1) atomicOr(&p.body[mt.c].err, 1);
        }
    }
    const TileBox tb = mark_points(p, cd, B, X, mt.count, lane);
    if (lane == 0) p.tbox[tix] = tb;
    if (dl > 0.0) {
        const double Y[3] = {X[0] + dl * N[0], X[1] + dl * N[1], X[2] + dl * N[2]};
        const TileBox to = mark_points(p, cd, B, Y, mt.count, lane);
        if (lane == 0) p.tbox[n_mtiles + tix] = to;   // the force-surface points' box
    }
}

// Per-marker epilogue of the l = 0 interpolation: plain start, features and
// the stress-integral parts into o[kPart] (vin = interpolated rho - 1, u*,
// sigma; o may alias vin).  h_k becomes h0 when the first spread has been
// done (spread set), else 0.
__device__ inline void force_epilogue(const DevPtrs &p, int k, const BodyView &B, const double *vin, double *o,
                                      int spread)
{
    double v[kRegFields];
#pragma unroll
    for (int f = 0; f < kRegFields; f++) v[f] = vin[f];
    const double X[3] = {p.X[3 * k], p.X[3 * k + 1], p.X[3 * k + 2]};
    const double pr = (double)CS2 * v[0];
    const double sg[3][3] = {{v[4], v[7], v[8]}, {v[7], v[5], v[9]}, {v[8], v[9], v[6]}};
    const double nk[3] = {p.N[3 * k], p.N[3 * k + 1], p.N[3 * k + 2]};
    const double dS = p.dS[k];
    double s[3], rel[3], ts[3], h0[3], hp[3], hq[3], h0q[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        h0[a] = p.U[3 * k + a] - v[1 + a];
        hp[a] = p.hk[3 * k + a];    // the previous step's final h
        hq[a] = p.hk2[3 * k + a];   // the final h of the step before
        h0q[a] = p.h0[3 * k + a];   // the previous step's plain start
    }
    // warm-start features: the plain start U - I[u*] (an invertible linear
    // map of I[u*] and U that keeps their small difference out of
    // cancellation), h(t-1), and the changes h(t-1) - h(t-2) and
    // h0(t) - h0(t-1), over the marker's scale |h0| + |h(t-1)|; the normal
    // and the area
    const double sc = fmax(sqrt(h0[0] * h0[0] + h0[1] * h0[1] + h0[2] * h0[2]) +
                               sqrt(hp[0] * hp[0] + hp[1] * hp[1] + hp[2] * hp[2]), 1e-14);
    p.hs[k] = sc;
    float *ft = p.feat + (long long)kMlpIn * k;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        s[a] = sg[a][0] * nk[0] + sg[a][1] * nk[1] + sg[a][2] * nk[2];
        rel[a] = X[a] - B.r[a];
        ft[kFeatH0 + a] = (float)(h0[a] / sc);
        ft[kFeatHPrev + a] = (float)(hp[a] / sc);
        ft[kFeatDH + a] = (float)((hp[a] - hq[a]) / sc);
        ft[kFeatDH0 + a] = (float)((h0[a] - h0q[a]) / sc);
        ft[kFeatNormal + a] = (float)nk[a];
        if (a == 0) ft[kFeatArea] = (float)dS;
        // h_k holds what has been spread so far; dh is the next increment
        p.hk2[3 * k + a] = hp[a];
        p.h0[3 * k + a] = h0[a];
        p.hk[3 * k + a] = spread ? 0.0 + h0[a] : 0.0;
        p.dh[3 * k + a] = h0[a];
    }
    cross3(rel, s, ts);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        o[a] = dS * s[a];
        o[3 + a] = dS * ts[a];
        o[6 + a] = dS * (-pr) * nk[a];
    }
}

// Tile sums of the per-marker parts (the first kPart entries of each row of
// tp, a row per marker), in marker order (deterministic).
template <int W>
__device__ inline void tile_part_sum(const DevPtrs &p, int tix, int count, const double (*tp)[W])
{
    __syncthreads();
    if ((int)threadIdx.x < kPart) {
        double acc = 0.0;
        for (int j = 0; j < count; j++) acc += tp[j][threadIdx.x];
        p.part[(long long)kPart * tix + threadIdx.x] = acc;
    }
}

// Case totals of the per-tile force, torque and pressure-force parts, in a
// fixed order: strided per-thread sums over the case's tiles, a fixed
// butterfly inside each wavefront, then the wavefronts in order.
__device__ inline void case_force_total(const DevPtrs &p, const CaseDev &cd, BodyDev &B)
{
    __shared__ double sh[4][kPart];
    double acc[kPart];
#pragma unroll
    for (int j = 0; j < kPart; j++) acc[j] = 0.0;
    for (int t = threadIdx.x; t < cd.n_tiles; t += blockDim.x) {
        const double *o = p.part + (long long)kPart * (cd.tile_off + t);
#pragma unroll
        for (int j = 0; j < kPart; j++) acc[j] += o[j];
    }
#pragma unroll
    for (int j = 0; j < kPart; j++) acc[j] = wave_sum(acc[j]);
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < kPart; j++) sh[wave][j] = acc[j];
    __syncthreads();
    if (threadIdx.x < kPart) {
        double v = 0.0;
        for (int w = 0; w < nw; w++) v += sh[w][threadIdx.x];
        double *dst = threadIdx.x < 3 ? &B.F[threadIdx.x] : (threadIdx.x < 6 ? &B.T[threadIdx.x - 3] : &B.Fp[threadIdx.x - 6]);
        *dst = v;
    }
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Case maximum of the per-tile residuals into resid and resid_hist[slot].
__device__ inline void case_resid_total(const DevPtrs &p, const CaseDev &cd, BodyDev &B, int slot)
{
    __shared__ double sh[4];
    double m = 0.0;
    for (int t = threadIdx.x; t < cd.n_tiles; t += blockDim.x) m = fmax(m, p.res[cd.tile_off + t]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) v = fmax(v, sh[w]);
        B.resid = v;
        if (slot >= 0 && slot < 16) B.resid_hist[slot] = v;
    }
}

// Spread of one marker's increment d (held by every lane) through the lane's
// stencil node with weight W dS_k: fixed point, into the tile's LDS
// accumulator (box cell i) or, when the box does not fit, straight into the
// region accumulator Hc (region cell q, -1 outside).
__device__ inline void spread_node(const DevPtrs &p, int c, const TileBox &tb, int i, int q, double wS,
                                   const double d[3], unsigned long long (*acc)[kBoxCells], long long *Hc, int L3)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double v = d[a] * wS;
        long long fx = 0;
        if (fabs(v) < 1.0e6) fx = __double2ll_rn(v * kFixScale);
        else atomicOr(&p.body[c].err, 2);
        if (tb.fits) atomicAdd(&acc[a][i], (unsigned long long)fx);
        else if (q >= 0) atomicAdd((unsigned long long *)&Hc[a * L3 + q], (unsigned long long)fx);
    }
}

// The tile's LDS accumulator into the region accumulator: one global atomic
// per touched cell and component (after a barrier).
__device__ inline void spread_flush(const TileBox &tb, int ncell, int L, int L3,
                                    const unsigned long long (*acc)[kBoxCells], long long *Hc)
{
    for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
        const int q = box_region_cell(i, tb, L);
#pragma unroll
        for (int a = 0; a < 3; a++)
            if (acc[a][i] != 0ull) atomicAdd((unsigned long long *)&Hc[a * L3 + q], acc[a][i]);
    }
}

// Entry f of marker k's record: X (0..2), U (3..5), dS (6), the stencil
// weights (7..18), h_k (19..21).  The force kernel keeps entries 0..18.
constexpr int kRecW = 7, kRecH = 19, kRecForce = 19, kRecUpdate = 22;

// The tile kernels of the coupling run beside the lattice kernel, whose waves
// each hold 64 VGPRs and 96 SGPRs and fill every wave slot of a SIMD.  A
// coupling wave starts only in a slot a lattice wave frees, so the force and
// update passes come in two register budgets, MINW = 8 waves per SIMD (the
// lattice kernel's own budget) and MINW = 1 (registers as the LDS-bound
// occupancy allows).
// FP32 storage takes the first: measured at the 256 x 256 x 768 case, its
// coupling then runs during the lattice kernel instead of after it, 50 us
// less per step.  With FP16 storage the coupling already runs beside the
// lattice kernel and the tighter budget only slows that kernel, so the
// reduced-precision and moment stores take the second.  The LDS of these
// kernels is taken at launch (dynamic), so that the compiler's occupancy
// target is set by the register budget and not by the LDS size; the layouts
// are carved below, 8-byte arrays first.

struct LdsCarve {
    unsigned char *at;
    template <class A>
    __device__ A &take()
    {
        A &r = *reinterpret_cast<A *>(at);
        at += sizeof(A);
        return r;
    }
};

constexpr size_t kLdsForce = sizeof(unsigned long long[3][kBoxCells]) + sizeof(double[kTileMarkers][kRegFields]) +
                             sizeof(double[kTileMarkers][kRecForce]) + sizeof(double[kTileMarkers][3]) +
                             sizeof(float[kRegFields][kBoxCells]);
constexpr size_t kLdsUpdate = sizeof(double[3][kBoxCells]) + sizeof(unsigned long long[3][kBoxCells]) +
                              sizeof(double[kTileMarkers][kRecUpdate]) + sizeof(double[kTileMarkers][3]) +
                              sizeof(double[kTileMarkers]);
static_assert(kLdsForce <= 65536 && kLdsUpdate <= 65536, "tile kernel LDS");
// Waves per SIMD that the LDS of a 256-thread workgroup allows (160 KB per
// CU): the occupancy the unconstrained budget is compiled for, as with static
// LDS.
constexpr int lds_waves(size_t bytes) { return (int)std::min<size_t>(8, (160 * 1024) / bytes); }
__device__ inline double marker_record(const DevPtrs &p, int k, int f)
{
    if (f < 3) return p.X[3 * k + f];
    if (f < 6) return p.U[3 * k + f - 3];
    if (f == 6) return p.dS[k];
    if (f < kRecH) return p.wt[12 * k + f - kRecW];
    return p.hk[3 * k + f - kRecH];
}

// A tile's marker records into LDS (row j = marker first + j), in two loads
// per thread issued together; the caller stores them after its other loads
// and before its barrier.
template <int NREC>
struct RecordLoad {
    static_assert(kTileMarkers * NREC <= 512, "two loads per thread of a 256-thread workgroup");
    double v[2];
    __device__ inline void load(const DevPtrs &p, const MarkerTile &mt)
    {
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int t = (int)threadIdx.x + 256 * u;
            v[u] = t < mt.count * NREC ? marker_record(p, mt.first + t / NREC, t % NREC) : 0.0;
        }
    }
    __device__ inline void store(const MarkerTile &mt, double (*rec)[NREC]) const
    {
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int t = (int)threadIdx.x + 256 * u;
            if (t < mt.count * NREC) rec[t / NREC][t % NREC] = v[u];
        }
    }
};

// Spread of the tile's per-marker increments d[j] (LDS rows) after a
// barrier: wavefront w takes markers w, w+4, ...; lane l is stencil node l,
// so the 64 LDS atomics of one instruction go to 64 different cells.
__device__ inline void spread_tile(const DevPtrs &p, const MarkerTile &mt, const TileBox &tb, const CaseDev &cd,
                                   const BodyView &B, const double *rbase, int nrec, const double (*d)[3],
                                   unsigned long long (*acc)[kBoxCells], long long *Hc, int L3)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = wave; j < mt.count; j += blockDim.x >> 6) {
        const double *rc = rbase + j * nrec;
        const double X[3] = {rc[0], rc[1], rc[2]};
        double W;
        int i = 0, q = -1;
        if (tb.fits) {
            i = box_node_w(X, rc + kRecW, lane, tb, W);
        } else {
            const Node nd = stencil_node(X, lane, cd, B);
            W = nd.W;
            q = nd.q;
        }
        spread_node(p, mt.c, tb, i, q, W * rc[6], d[j], acc, Hc, L3);
    }
}

// l = 0 and the stress integral over a tile (a row of 16 lanes per marker).
// With spread set, also the first forcing cycle's spread of the plain start
// h0 into accumulator 0 (h_k = h0).
template <int MINW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MINW, MINW == 8 ? 8 : lds_waves(kLdsForce))))
k_interp_force_tiles(DevPtrs p, int n_mtiles, int spread)
{
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    LdsCarve lc{lds_dyn};
    auto &acc = lc.take<unsigned long long[3][kBoxCells]>();
    auto &ep = lc.take<double[kTileMarkers][kRegFields]>();    // interpolated fields, then the marker's parts
    auto &mrec = lc.take<double[kTileMarkers][kRecForce]>();   // the tile's marker records
    auto &dinc = lc.take<double[kTileMarkers][3]>();           // the markers' increments (h0) to spread
    auto &box = lc.take<float[kRegFields][kBoxCells]>();
    const int tix = tile_of_block((int)blockIdx.x, n_mtiles);
    if (tix >= n_mtiles) return;
    const MarkerTile mt = p.mtiles[tix];
    const CaseDev cd = p.cases[mt.c];
    const BodyView B = body_view(p.body[mt.c]);
    if (B.err != 0) return;
    const int L = cd.L, L3 = L * L * L;
    const float *R = p.reg + cd.reg_off * kRegFields;
    long long *H0 = p.H + cd.reg_off * 3;
    const TileBox tb = p.tbox[tix];
    const int ncell = tb.e[0] * tb.e[1] * tb.e[2];
    // the markers' records load in the same round as the box
    RecordLoad<kRecForce> rl;
    rl.load(p, mt);
    if (tb.fits) {
        for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
            const int q = box_region_cell(i, tb, L);
#pragma unroll
            for (int f = 0; f < kRegFields; f++) box[f][i] = R[f * L3 + q];
            acc[0][i] = acc[1][i] = acc[2][i] = 0ull;
        }
    }
    rl.store(mt, mrec);
    __syncthreads();
    // rows past the tile's markers repeat marker 0 and store nothing
    const int j = threadIdx.x >> 4, col = threadIdx.x & 15;
    const bool on = j < mt.count;
    const double *rc = mrec[on ? j : 0];
    const double X[3] = {rc[0], rc[1], rc[2]};
    const Column cn = column_nodes(X, rc + kRecW, col, tb, cd, B);
    double v[kRegFields];
#pragma unroll
    for (int f = 0; f < kRegFields; f++) v[f] = 0.0;
#pragma unroll
    for (int z = 0; z < 4; z++) {
        if (tb.fits) {
#pragma unroll
            for (int f = 0; f < kRegFields; f++) v[f] += cn.W[z] * (double)box[f][cn.i[z]];
        } else if (cn.q[z] >= 0) {
#pragma unroll
            for (int f = 0; f < kRegFields; f++) v[f] += cn.W[z] * (double)R[f * L3 + cn.q[z]];
        }
    }
#pragma unroll
    for (int f = 0; f < kRegFields; f++) v[f] = row_sum(v[f]);
    if (on && col == 0) {
#pragma unroll
        for (int f = 0; f < kRegFields; f++) ep[j][f] = v[f];
#pragma unroll
        for (int a = 0; a < 3; a++) dinc[j][a] = rc[3 + a] - v[1 + a];
    }
    __syncthreads();
    if (spread) spread_tile(p, mt, tb, cd, B, &mrec[0][0], kRecForce, dinc, acc, H0, L3);
    // the tile's epilogues side by side, one thread per marker
    if ((int)threadIdx.x < mt.count) force_epilogue(p, mt.first + threadIdx.x, B, ep[threadIdx.x], ep[threadIdx.x], spread);
    tile_part_sum(p, tix, mt.count, ep);
    if (spread && tb.fits) spread_flush(tb, ncell, L, L3, acc, H0);
}

// Force surface variant: the stress integral on the parallel surface at
// distance force_offset outside the markers (points Y_k = X_k + delta n_k,
// same normals, areas dSo).  One workgroup per marker tile, as the force
// kernel: the box of the tile's surface-point stencils (from k_markers) is
// staged in LDS with rho - 1 and sigma, a row of 16 lanes per marker sums
// its stencil, one thread per marker forms its parts.  Overwrites the
// tile's force, torque and pressure-force sums written by the tile kernel.
__global__ void __launch_bounds__(256) k_offset_force(DevPtrs p, int n_mtiles)
{
    __shared__ float box[7][kBoxCells];
    __shared__ double ev[kTileMarkers][7];
    __shared__ double tp[kTileMarkers][kPart];
    const int tix = tile_of_block((int)blockIdx.x, n_mtiles);
    if (tix >= n_mtiles) return;
    const MarkerTile mt = p.mtiles[tix];
    const CaseDev cd = p.cases[mt.c];
    const BodyView B = body_view(p.body[mt.c]);
    if (B.err != 0 || !(cd.force_offset > 0.0)) return;
    const int L = cd.L, L3 = L * L * L;
    const float *R = p.reg + cd.reg_off * kRegFields;
    const TileBox tb = p.tbox[n_mtiles + tix];
    const int ncell = tb.e[0] * tb.e[1] * tb.e[2];
    // fields 0 (rho - 1) and 4..9 (sigma xx yy zz xy xz yz)
    if (tb.fits) {
        for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
            const int q = box_region_cell(i, tb, L);
            box[0][i] = R[q];
#pragma unroll
            for (int f = 1; f < 7; f++) box[f][i] = R[(f + 3) * L3 + q];
        }
    }
    __syncthreads();
    const int j = threadIdx.x >> 4, col = threadIdx.x & 15;
    const bool on = j < mt.count;
    const int k = mt.first + (on ? j : 0);
    const double dl = cd.force_offset;
    double Y[3], w[12];
#pragma unroll
    for (int a = 0; a < 3; a++) Y[a] = p.X[3 * k + a] + dl * p.N[3 * k + a];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int n0 = (int)floor(Y[d]) - 1;
#pragma unroll
        for (int o = 0; o < 4; o++) w[4 * d + o] = phi4((double)(n0 + o) - Y[d]);
    }
    const Column cn = column_nodes(Y, w, col, tb, cd, B);
    double v[7];
#pragma unroll
    for (int f = 0; f < 7; f++) v[f] = 0.0;
#pragma unroll
    for (int z = 0; z < 4; z++) {
        if (tb.fits) {
#pragma unroll
            for (int f = 0; f < 7; f++) v[f] += cn.W[z] * (double)box[f][cn.i[z]];
        } else if (cn.q[z] >= 0) {
#pragma unroll
            for (int f = 0; f < 7; f++) v[f] += cn.W[z] * (double)R[(f == 0 ? 0 : f + 3) * L3 + cn.q[z]];
        }
    }
#pragma unroll
    for (int f = 0; f < 7; f++) v[f] = row_sum(v[f]);
    if (on && col == 0)
#pragma unroll
        for (int f = 0; f < 7; f++) ev[j][f] = v[f];
    __syncthreads();
    if ((int)threadIdx.x < mt.count) {
        const int m = mt.first + threadIdx.x;
        const double *e = ev[threadIdx.x];
        const double nk[3] = {p.N[3 * m], p.N[3 * m + 1], p.N[3 * m + 2]};
        const double pr = (double)CS2 * e[0];
        const double sg[3][3] = {{e[1], e[4], e[5]}, {e[4], e[2], e[6]}, {e[5], e[6], e[3]}};
        double s[3], rel[3], ts[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            s[a] = sg[a][0] * nk[0] + sg[a][1] * nk[1] + sg[a][2] * nk[2];
            rel[a] = p.X[3 * m + a] + dl * nk[a] - B.r[a];
        }
        cross3(rel, s, ts);
        const double dA = p.dSo[m];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            tp[threadIdx.x][a] = dA * s[a];
            tp[threadIdx.x][3 + a] = dA * ts[a];
            tp[threadIdx.x][6 + a] = dA * (-pr) * nk[a];
        }
    }
    tile_part_sum(p, tix, mt.count, tp);
}

// Spreading of the increments dh over a tile into accumulator 0 (H += S[dh],
// h_k += dh): LDS accumulation, then one HBM atomic per touched cell.  With
// masked set, cases whose sequence has ended are skipped.
__global__ void __launch_bounds__(256) k_spread_tiles(DevPtrs p, int n_mtiles, int masked)
{
    __shared__ unsigned long long acc[3][kBoxCells];
    __shared__ double mrec[kTileMarkers][kRecForce];   // the tile's marker records
    __shared__ double dinc[kTileMarkers][3];           // the increments dh to spread
    const int tix = tile_of_block((int)blockIdx.x, n_mtiles);
    if (tix >= n_mtiles) return;
    const MarkerTile mt = p.mtiles[tix];
    const CaseDev cd = p.cases[mt.c];
    const BodyView B = body_view(p.body[mt.c]);
    if (B.err != 0 || (masked && !B.active)) return;
    const int L = cd.L, L3 = L * L * L;
    long long *H = p.H + cd.reg_off * 3;
    const TileBox tb = p.tbox[tix];
    const int ncell = tb.e[0] * tb.e[1] * tb.e[2];
    RecordLoad<kRecForce> rl;
    rl.load(p, mt);
    // thread j < count: marker j's increment, and h_k += dh
    const int t = threadIdx.x;
    double dh[3] = {0.0, 0.0, 0.0}, hk[3] = {0.0, 0.0, 0.0};
    if (t < mt.count)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            dh[a] = p.dh[3 * (mt.first + t) + a];
            hk[a] = p.hk[3 * (mt.first + t) + a];
        }
    if (tb.fits)
        for (int i = threadIdx.x; i < ncell; i += blockDim.x) acc[0][i] = acc[1][i] = acc[2][i] = 0ull;
    rl.store(mt, mrec);
    if (t < mt.count)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            dinc[t][a] = dh[a];
            p.hk[3 * (mt.first + t) + a] = hk[a] + dh[a];
        }
    __syncthreads();
    spread_tile(p, mt, tb, cd, B, &mrec[0][0], kRecForce, dinc, acc, H, L3);
    __syncthreads();
    if (tb.fits) spread_flush(tb, ncell, L, L3, acc, H);
}

// Interpolation of u* + H over a tile (staged in LDS, FP64; H the sum of
// accumulators 0 .. NB-1), the residual U_k - I[u* + H](X_k), the next
// increment dh = that residual, and the tile's largest residual component.
// With spread_to >= 0 the same pass spreads dh (the next cycle's spread,
// h_k += dh) into accumulator spread_to, which no interpolation of this
// pass reads.
template <int NB, int MINW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MINW, MINW == 8 ? 8 : lds_waves(kLdsUpdate))))
k_interp_update_tiles(DevPtrs p, int n_mtiles, int masked, int spread_to, int ft_total)
{
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    LdsCarve lc{lds_dyn};
    auto &box = lc.take<double[3][kBoxCells]>();
    auto &acc = lc.take<unsigned long long[3][kBoxCells]>();
    auto &mrec = lc.take<double[kTileMarkers][kRecUpdate]>();   // the tile's marker records
    auto &dinc = lc.take<double[kTileMarkers][3]>();            // the markers' increments e to spread
    auto &rmax = lc.take<double[kTileMarkers]>();
    const int tix = tile_of_block((int)blockIdx.x, n_mtiles);
    if (tix >= n_mtiles) return;
    const MarkerTile mt = p.mtiles[tix];
    const CaseDev cd = p.cases[mt.c];
    const BodyView B = body_view(p.body[mt.c]);
    if (B.err != 0 || (masked && !B.active)) return;
    const int L = cd.L, L3 = L * L * L;
    const float *R = p.reg + cd.reg_off * kRegFields;
    const long long *H = p.H + cd.reg_off * 3;
    long long *Hs = p.H + (spread_to > 0 ? spread_to : 0) * p.hstride + cd.reg_off * 3;
    const TileBox tb = p.tbox[tix];
    const int ncell = tb.e[0] * tb.e[1] * tb.e[2];
    // H at region cell q and component a: the exact integer sum of the accumulators
    const long long hstride = p.hstride;
    auto h_at = [&](int a, int q) {
        long long h = H[a * L3 + q];
#pragma unroll
        for (int b = 1; b < NB; b++) h += H[b * hstride + a * L3 + q];
        return h;
    };
    // the markers' records load in the same round as the box
    RecordLoad<kRecUpdate> rl;
    rl.load(p, mt);
    if (tb.fits) {
        for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
            const int q = box_region_cell(i, tb, L);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                box[a][i] = (double)R[(1 + a) * L3 + q] + (double)h_at(a, q) * kFixInv;
                acc[a][i] = 0ull;
            }
        }
    }
    rl.store(mt, mrec);
    __syncthreads();
    // rows past the tile's markers repeat marker 0 and store nothing
    const int j = threadIdx.x >> 4, col = threadIdx.x & 15;
    const bool on = j < mt.count;
    const double *rc = mrec[on ? j : 0];
    const double X[3] = {rc[0], rc[1], rc[2]};
    const Column cn = column_nodes(X, rc + kRecW, col, tb, cd, B);
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int z = 0; z < 4; z++) {
        if (tb.fits) {
#pragma unroll
            for (int a = 0; a < 3; a++) v[a] += cn.W[z] * box[a][cn.i[z]];
        } else if (cn.q[z] >= 0) {
            const int q = cn.q[z];
#pragma unroll
            for (int a = 0; a < 3; a++)
                v[a] += cn.W[z] * ((double)R[(1 + a) * L3 + q] + (double)h_at(a, q) * kFixInv);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; a++) v[a] = row_sum(v[a]);
    const double e[3] = {rc[3] - v[0], rc[4] - v[1], rc[5] - v[2]};
    if (on && col == 0) {
        const int k = mt.first + j;
        double res = 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            res = fmax(res, fabs(e[a]));
            p.dh[3 * k + a] = e[a];
            if (spread_to >= 0) p.hk[3 * k + a] = rc[kRecH + a] + e[a];
            dinc[j][a] = e[a];
        }
        rmax[j] = res;
    }
    __syncthreads();
    if (spread_to >= 0) spread_tile(p, mt, tb, cd, B, &mrec[0][0], kRecUpdate, dinc, acc, Hs, L3);
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int t = 0; t < mt.count; t++) m = fmax(m, rmax[t]);
        p.res[tix] = m;
    }
    if (spread_to >= 0 && tb.fits) spread_flush(tb, ncell, L, L3, acc, Hs);
    // the case's force totals from the force kernels' tile parts (complete at
    // this kernel's start), formed by the workgroup of its first tile
    if (ft_total && tix == cd.tile_off) case_force_total(p, cd, p.body[mt.c]);
}

// FP64 force, torque and pressure-force totals of each case from its tile
// parts (one 256-thread workgroup per case, fixed order).
__global__ void __launch_bounds__(256) k_reduce_ft(DevPtrs p)
{
    const int c = blockIdx.x;
    const CaseDev &cd = p.cases[c];
    if (cd.M == 0 || p.body[c].err != 0) return;
    case_force_total(p, cd, p.body[c]);
}

// Max residual over the tiles of a case: into resid and resid_hist[slot].
// With masked set only cases still active are reduced; with gate_cycle > 0
// (a learned-start cycle) a case whose residual is at or below its gate is
// accepted and leaves the sequence.
__global__ void __launch_bounds__(256) k_reduce_resid(DevPtrs p, int slot, int masked, int gate_cycle)
{
    const int c = blockIdx.x;
    const CaseDev &cd = p.cases[c];
    BodyDev &B = p.body[c];
    if (cd.M == 0 || B.err != 0 || (masked && !B.active)) return;
    case_resid_total(p, cd, B, slot);
    if (threadIdx.x == 0 && gate_cycle > 0 && B.resid <= B.gate) {
        B.active = 0;
        B.accepts += 1;
        B.warm_cyc_sum += gate_cycle;
    }
}

// Start of a learned-start sequence: every live case runs cycles.
__global__ void k_gate_begin(DevPtrs p, int n_cases)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cases) return;
    BodyDev &B = p.body[c];
    B.active = 1;
    B.fallback = 0;
}

// End of the learned-start cycles: a case not accepted within them falls
// back to the plain start and stays active for the plain cycles.
__global__ void k_gate(DevPtrs p, int n_cases)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cases) return;
    BodyDev &B = p.body[c];
    if (p.cases[c].M == 0 || B.err != 0) return;
    B.fallback = B.active;
    if (B.fallback) B.rejects += 1;
}

// Warm start without a network: the previous step's final h_k (kept in the
// features over the marker's scale).
__global__ void k_warm_previous(DevPtrs p, int Mtot)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mtot || p.body[p.mcase[k]].err != 0) return;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double h = (double)p.feat[(long long)kMlpIn * k + kFeatHPrev + a] * p.hs[k];
        p.hk[3 * k + a] = 0.0;
        p.dh[3 * k + a] = h;
    }
}

// Fallback preparation: plain start h_k = U_k - I[u*](X_k) ...
__global__ void k_fallback_markers(DevPtrs p, int Mtot)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mtot) return;
    const BodyDev &B = p.body[p.mcase[k]];
    if (B.err != 0 || !B.fallback) return;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        p.hk[3 * k + a] = 0.0;
        p.dh[3 * k + a] = p.h0[3 * k + a];
    }
}

// ... and an empty immersed-force accumulator.
__global__ void k_fallback_zero(DevPtrs p)
{
    const int c = blockIdx.y;
    const CaseDev &cd = p.cases[c];
    const BodyDev &B = p.body[c];
    if (cd.M == 0 || B.err != 0 || !B.fallback) return;
    const int L3 = cd.L * cd.L * cd.L;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= L3 || !p.mark[cd.reg_off + q]) return;
    long long *H = p.H + cd.reg_off * 3;
#pragma unroll
    for (int j = 0; j < kHBufs; j++) {
        H[j * p.hstride + q] = 0;
        H[j * p.hstride + L3 + q] = 0;
        H[j * p.hstride + 2 * L3 + q] = 0;
    }
}

// Training targets: the final h_k minus the previous step's h, over the
// marker's feature scale: h_k / s_k - feature 9..11.
__global__ void k_targets(DevPtrs p, int Mtot, float *out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mtot) return;
    const float *ft = p.feat + (long long)kMlpIn * k;
#pragma unroll
    for (int a = 0; a < 3; a++) out[3 * k + a] = (float)(p.hk[3 * k + a] / p.hs[k] - (double)ft[kFeatHPrev + a]);
}

// Forced collision of Sec. 2.2: the lattice kernel wrote
// f0(rho, u) + (1 - 1/tau) f1; cells carrying an immersed force get
// f0(rho, u + tau h) - f0(rho, u) added (in the momentum-exact variant less
// the first-order term w_i xi_i . (tau - 1) rho h / cs^2).  Only cells
// marked this step can carry a force; their marks are cleared here.
template <class CD>
__global__ void k_correct(typename CD::T *__restrict__ cur, DevPtrs p, int did, int resid_slot)
{
    const int c = blockIdx.y;
    const CaseDev cd = p.cases[c];
    const BodyView B = body_view(p.body[c]);
    if (cd.M == 0 || B.err != 0) return;
    // the forcing sequence's residual (its tile maxima are complete here)
    if (resid_slot >= 0 && blockIdx.x == 0) case_resid_total(p, cd, p.body[c], resid_slot);
    const int L = cd.L, L3 = L * L * L;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= L3) return;
    unsigned char &mk = p.mark[cd.reg_off + q];
    if (!mk) return;
    mk = 0;
    const int a = q % L, b = (q / L) % L, cc = q / (L * L);
    const int gz = B.org[2] + cc;
    if (gz < 0 || gz >= cd.nz) return;
    const int gx = wrapi(B.org[0] + a, cd.nx), gy = wrapi(B.org[1] + b, cd.ny);
    int zc = gz + B.z0;
    if (zc >= cd.nz) zc -= cd.nz;
    const int off = (zc * cd.ny + gy) * cd.nx + gx;
    typename CD::T *dst = cur + cd.pop_off;
    // the accumulators, the fields and the populations in one round of loads
    const long long *H = p.H + cd.reg_off * 3;
    const float *R = p.reg + cd.reg_off * kRegFields;
    long long h0 = 0, h1 = 0, h2 = 0;
#pragma unroll
    for (int j = 0; j < kHBufs; j++) {
        h0 += H[j * p.hstride + q];
        h1 += H[j * p.hstride + L3 + q];
        h2 += H[j * p.hstride + 2 * L3 + q];
    }
    const float rho = 1.0f + R[q];
    const float u[3] = {R[L3 + q], R[2 * L3 + q], R[3 * L3 + q]};
    // a cell of the full-precision box is corrected there (FP32) and stored
    // rounded once; elsewhere the stored value is decoded and re-rounded
    int slot = -1;
    float *F = nullptr;
    long long fplane = 0;
    if (cd.LB[0] > 0 && p.body[c].fvalid[did]) {
        const BodyDev &Bd = p.body[c];
        const int fo[3] = {Bd.fo[did][0], Bd.fo[did][1], Bd.fo[did][2]};
        slot = fine_slot(cd, fo, gx, gy, gz);
        F = p.fine[did] + cd.fine_off;
        fplane = fine_plane(cd);
    }
    float g[Q];
    if (slot >= 0) {
#pragma unroll
        for (int i = 0; i < Q; i++) g[i] = F[(long long)i * fplane + slot];
    } else {
        Unroll<0, Q>::run([&](auto I) {
            constexpr int i = decltype(I)::value;
            g[i] = CD::template dec<i>(dst[(long long)i * cd.plane + off]);
        });
    }
    if ((h0 | h1 | h2) == 0) return;
    const float tau = tau_at(cd.tau0, cd.nz, cd.sponge, gz);
    const float us[3] = {u[0] + tau * (float)((double)h0 * kFixInv), u[1] + tau * (float)((double)h1 * kFixInv),
                         u[2] + tau * (float)((double)h2 * kFixInv)};
    float A[Q], d[Q];
    shift_coeffs(rho, u, us, A);
    if (cd.forcing == 1) {
        // momentum-exact variant: the first-order coefficients (m = e_x, e_y,
        // e_z) become rho h instead of rho tau h
        const float k = (tau - 1.0f) * rho;
        A[1] -= k * (float)((double)h0 * kFixInv);
        A[3] -= k * (float)((double)h1 * kFixInv);
        A[9] -= k * (float)((double)h2 * kFixInv);
    }
    hermite_to_populations(A, d);
    Unroll<0, Q>::run([&](auto I) {
        constexpr int i = decltype(I)::value;
        const float v = g[i] + d[i];
        if constexpr (!std::is_same<CD, CodecF32>::value)
            if (slot >= 0) F[(long long)i * fplane + slot] = v;
        dst[(long long)i * cd.plane + off] = CD::template enc<i>(v);
    });
}

// The forced correction on moment storage: the stored moments stay the
// regularized state; the shift of every cell of the particle region goes to
// the case's forcing box, (tau h, lambda) on forced cells and zero elsewhere,
// with lambda = 1, or 1 / tau in the momentum-exact variant (the first-order
// term then carries rho h).  The box's origin is recorded in ring-slot
// coordinates, which a window shift leaves in place.  Marks are cleared.
__global__ void k_correct_mom(DevPtrs p, int resid_slot)
{
    const int c = blockIdx.y;
    const CaseDev cd = p.cases[c];
    const BodyView B = body_view(p.body[c]);
    if (cd.M == 0 || B.err != 0) return;
    if (resid_slot >= 0 && blockIdx.x == 0) case_resid_total(p, cd, p.body[c], resid_slot);
    const int L = cd.L, L3 = L * L * L;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        BodyDev &Bw = p.body[c];
        Bw.dorg[0] = wrapi(B.org[0], cd.nx);
        Bw.dorg[1] = wrapi(B.org[1], cd.ny);
        Bw.dorg[2] = wrapi(B.org[2] + B.z0, cd.nz);
        Bw.dvalid = 1;
    }
    if (q >= L3) return;
    float *D = p.dsh + cd.reg_off * 4;
    float sh[4] = {0.0f, 0.0f, 0.0f, 1.0f};
    unsigned char &mk = p.mark[cd.reg_off + q];
    const int gz = B.org[2] + q / (L * L);
    if (mk && gz >= 0 && gz < cd.nz) {
        const long long *H = p.H + cd.reg_off * 3;
        long long h0 = 0, h1 = 0, h2 = 0;
#pragma unroll
        for (int j = 0; j < kHBufs; j++) {
            h0 += H[j * p.hstride + q];
            h1 += H[j * p.hstride + L3 + q];
            h2 += H[j * p.hstride + 2 * L3 + q];
        }
        const float tau = tau_at(cd.tau0, cd.nz, cd.sponge, gz);
        sh[0] = tau * (float)((double)h0 * kFixInv);
        sh[1] = tau * (float)((double)h1 * kFixInv);
        sh[2] = tau * (float)((double)h2 * kFixInv);
        if (cd.forcing == 1) sh[3] = 1.0f / tau;
    }
    if (mk) mk = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) D[k * (long long)L3 + q] = sh[k];
}

// ----------------------------------------------------------------- window
// Sec. 2.5: below h_end the content and the body move up by dz rows.  With
// the ring layout the move is the origin change z0 -> z0 - dz; the dz rows
// that now form the bottom (the former top rows) restart at rest.
// The step's record for the case's log ring, taken after the window test.
struct StepRecord {
    double v[kLogFields];
};

__device__ inline StepRecord window_trigger_case(const DevPtrs &p, int c)
{
    const CaseDev &cd = p.cases[c];
    BodyDev &B = p.body[c];
    // the test's operands in one round of loads (no short-circuit)
    const int M = cd.M, dz = cd.dz, nz = cd.nz, err = B.err;
    const double h_end = cd.h_end, rz = B.r[2];
    const bool shift = (M > 0) & (err == 0) & (dz > 0) & (h_end > 0.0) & (rz < h_end);
    B.shift_now = 0;
    if (shift) {
        B.r[2] = rz + (double)dz;
        B.z0 = wrapi(B.z0 - dz, nz);
        B.fo[0][2] += dz;   // the full-precision boxes move with the content
        B.fo[1][2] += dz;
        B.shift_now = 1;
        B.shifts += 1;
    }
    StepRecord rec;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        rec.v[a] = B.r[a];
        rec.v[12 + a] = B.v[a];
        rec.v[15 + a] = B.w[a];
        rec.v[18 + a] = B.F[a];
        rec.v[21 + a] = B.T[a];
        rec.v[24 + a] = B.Fp[a];
    }
#pragma unroll
    for (int a = 0; a < 9; a++) rec.v[3 + a] = B.d[a];
    rec.v[27] = B.resid;
    rec.v[28] = B.steps;
    rec.v[29] = B.shifts;
    rec.v[30] = B.z0;
    rec.v[31] = B.err;
    return rec;
}

// Appends a record to the case's log ring.  Written last in its kernel: the
// stores go through a plain double pointer, which the compiler must assume
// may alias the body state, so no body field is read after them.
__device__ inline void log_append(const DevPtrs &p, int c, const StepRecord &rec)
{
    BodyDev &B = p.body[c];
    const unsigned int n = B.logged;
    B.logged = n + 1;
    double *dst = p.log + ((long long)c * kLogCap + n % kLogCap) * kLogFields;
#pragma unroll
    for (int k = 0; k < kLogFields; k++) dst[k] = rec.v[k];
}

__global__ void k_window_trigger(DevPtrs p, int n_cases)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cases) return;
    const StepRecord rec = window_trigger_case(p, c);
    log_append(p, c, rec);
}

// The end of one step and the start of the next in one launch, for steps
// the library sequences itself (lbm_run, graph capture): the window test of
// step t, then the body advance of step t + 1, then step t's record.  The
// window reset that follows reads no field the advance writes (it uses the
// ring origin and the full-precision box origins), so the result is that of
// the separate kernels, bit for bit.
__global__ void k_window_advance(DevPtrs p, int n_cases)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cases) return;
    const StepRecord rec = window_trigger_case(p, c);
    body_advance_case(p, c);
    log_append(p, c, rec);
}

template <class CD>
__global__ void k_window_reset(typename CD::T *__restrict__ cur, DevPtrs p, int cid)
{
    const int c = blockIdx.y;
    const CaseDev &cd = p.cases[c];
    const BodyDev &B = p.body[c];
    if (!B.shift_now) return;
    const int slab = cd.nx * cd.ny;
    // grid-strided: the launch stays small on the many steps without a shift
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < cd.dz * slab; idx += gridDim.x * blockDim.x) {
        const int zrow = idx / slab, rem = idx - zrow * slab;
        int zc = zrow + B.z0;
        if (zc >= cd.nz) zc -= cd.nz;
        typename CD::T *dst = cur + cd.pop_off + (long long)zc * slab + rem;
        if constexpr (std::is_same<CD, CodecMom>::value) {
#pragma unroll
            for (int k = 0; k < 10; k++) dst[(long long)k * cd.plane] = 0.0f;   // the rest state's moments
        } else {
            Unroll<0, Q>::run([&](auto I) {
                constexpr int i = decltype(I)::value;
                dst[(long long)i * cd.plane] = CD::template enc<i>(0.0f);
            });
            if (cd.LB[0] > 0 && B.fvalid[cid]) {
                const int slot = fine_slot(cd, B.fo[cid], rem % cd.nx, rem / cd.nx, zrow);
                if (slot >= 0) {
                    float *F = p.fine[cid] + cd.fine_off;
                    const long long fplane = fine_plane(cd);
#pragma unroll
                    for (int i = 0; i < Q; i++) F[(long long)i * fplane + slot] = 0.0f;
                }
            }
        }
    }
}

// --------------------------------------------------------------- launchers
hipError_t launch_body_advance(const DevPtrs &p, int n_cases, hipStream_t s)
{
    hipLaunchKernelGGL(k_body_advance, dim3((n_cases + 63) / 64), dim3(64), 0, s, p, n_cases);
    return hipGetLastError();
}

template <class CD>
static hipError_t ibm_impl(const void *prev, void *cur, const DevPtrs &p, int n_cases, int Mtot, int n_mtiles,
                           int maxL3, int cycles, int warm_mode, const _Float16 *th16, int warm_cycles, int diag,
                           int force_surface, int prev_id, hipStream_t s)
{
    using T = typename CD::T;
    const dim3 blk(256);
    const dim3 reg_grid((maxL3 + 255) / 256, n_cases);
    const dim3 tile_grid((n_mtiles + 7) / 8 * 8);
    const dim3 mark_grid((Mtot + 255) / 256);
    hipLaunchKernelGGL(k_markers, tile_grid, dim3(64), 0, s, p, n_mtiles);
    if constexpr (std::is_same<CD, CodecMom>::value) {
        int L = 1;
        while ((long long)L * L * L < maxL3) L++;
        const long long E3 = (long long)(L + 2) * (L + 2) * (L + 2);
        hipLaunchKernelGGL(k_region_expand_mom, dim3((unsigned)((E3 + 255) / 256), n_cases), blk, 0, s, (const T *)prev, p);
    }
    hipLaunchKernelGGL(k_region_gather<CD>, reg_grid, blk, 0, s, (const T *)prev, p, prev_id);
    // plain start with at most kHBufs cycles: each cycle's spread rides on
    // the pass before it (force + spread 1, update c + spread c + 1)
    static_assert(kHBufs == 4, "the launch below instantiates 1..4 accumulators");
    // register budget of the tile passes: 8 waves per SIMD (they fit the
    // slots the lattice kernel frees) for the population stores, whose
    // coupling runs beside that kernel; the occupancy the LDS allows for the
    // moment store
    constexpr int W = std::is_same<CD, CodecMom>::value ? 1 : 8;
    const int fused = ibm_fused(warm_mode, cycles);
    hipLaunchKernelGGL(k_interp_force_tiles<W>, tile_grid, blk, kLdsForce, s, p, n_mtiles, fused);
    if (force_surface) hipLaunchKernelGGL(k_offset_force, tile_grid, blk, 0, s, p, n_mtiles);
    // the fused sequence forms the force totals in its first update pass
    if (!fused) hipLaunchKernelGGL(k_reduce_ft, dim3(n_cases), blk, 0, s, p);
    // one sequence of multi-direct forcing cycles (Sec. 2.2, l = 1..4): spread
    // the increment, then interpolate and form the next increment; the
    // residual after the last spread is the sequence's residual
    auto sequence = [&](int ncyc, int slot0, int masked) {
        for (int cyc = 1; cyc <= ncyc; cyc++) {
            hipLaunchKernelGGL(k_spread_tiles, tile_grid, blk, 0, s, p, n_mtiles, masked);
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_interp_update_tiles<1, W>), tile_grid, blk, kLdsUpdate, s, p, n_mtiles, masked, -1, 0);
            if (diag || cyc == ncyc)
                hipLaunchKernelGGL(k_reduce_resid, dim3(n_cases), blk, 0, s, p, slot0 + cyc - 1, masked, 0);
        }
    };
    if (fused) {
        for (int cyc = 1; cyc <= cycles; cyc++) {
            const int to = cyc < cycles ? cyc : -1;
            // the first pass forms the force totals; the last pass's residual
            // is reduced by the forced correction (or, with diag, every
            // cycle's by its own kernel)
            const int ft = cyc == 1;
            switch (cyc) {
            case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_interp_update_tiles<1, W>), tile_grid, blk, kLdsUpdate, s, p, n_mtiles, 0, to, ft); break;
            case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_interp_update_tiles<2, W>), tile_grid, blk, kLdsUpdate, s, p, n_mtiles, 0, to, ft); break;
            case 3: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_interp_update_tiles<3, W>), tile_grid, blk, kLdsUpdate, s, p, n_mtiles, 0, to, ft); break;
            default: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_interp_update_tiles<4, W>), tile_grid, blk, kLdsUpdate, s, p, n_mtiles, 0, to, ft); break;
            }
            if (diag)
                hipLaunchKernelGGL(k_reduce_resid, dim3(n_cases), blk, 0, s, p, cyc - 1, 0, 0);
        }
        (void)cur;
        return hipGetLastError();
    }
    if (warm_mode != 0) {
        // learned (or previous-h) start: cycles until the case's residual is
        // at or below its gate, at most warm_cycles; the rest restart plain
        if (warm_mode == 2) {
            hipError_t e = launch_mlp_warm_start(th16, p, Mtot, s);   // the network lives in mlp.hip
            if (e != hipSuccess) return e;
        } else {
            hipLaunchKernelGGL(k_warm_previous, mark_grid, blk, 0, s, p, Mtot);
        }
        const dim3 case_grid((n_cases + 63) / 64), case_blk(64);
        hipLaunchKernelGGL(k_gate_begin, case_grid, case_blk, 0, s, p, n_cases);
        for (int cyc = 1; cyc <= warm_cycles; cyc++) {
            hipLaunchKernelGGL(k_spread_tiles, tile_grid, blk, 0, s, p, n_mtiles, 1);
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_interp_update_tiles<1, W>), tile_grid, blk, kLdsUpdate, s, p, n_mtiles, 1, -1, 0);
            hipLaunchKernelGGL(k_reduce_resid, dim3(n_cases), blk, 0, s, p, cyc - 1, 1, cyc);
        }
        hipLaunchKernelGGL(k_gate, case_grid, case_blk, 0, s, p, n_cases);
        hipLaunchKernelGGL(k_fallback_markers, mark_grid, blk, 0, s, p, Mtot);
        hipLaunchKernelGGL(k_fallback_zero, reg_grid, blk, 0, s, p);
        sequence(cycles, 8, 1);
    } else {
        sequence(cycles, 0, 0);
    }
    (void)cur;
    return hipGetLastError();
}

template <class CD>
static hipError_t correct_impl(void *cur, const DevPtrs &p, int n_cases, int maxL3, int cur_id, int resid_slot,
                               hipStream_t s)
{
    const dim3 reg_grid((maxL3 + 255) / 256, n_cases);
    hipLaunchKernelGGL(k_correct<CD>, reg_grid, dim3(256), 0, s, (typename CD::T *)cur, p, cur_id, resid_slot);
    return hipGetLastError();
}

hipError_t launch_correct(int storage, void *cur, const DevPtrs &p, int n_cases, int Mtot, int maxL3, int cur_id,
                          int resid_slot, hipStream_t s)
{
    if (Mtot == 0) return hipSuccess;
    switch (storage) {
    case ST_MOM:
        hipLaunchKernelGGL(k_correct_mom, dim3((maxL3 + 255) / 256, n_cases), dim3(256), 0, s, p, resid_slot);
        return hipGetLastError();
    case ST_F16: return correct_impl<CodecF16>(cur, p, n_cases, maxL3, cur_id, resid_slot, s);
    case ST_BF16: return correct_impl<CodecBF16>(cur, p, n_cases, maxL3, cur_id, resid_slot, s);
    default: return correct_impl<CodecF32>(cur, p, n_cases, maxL3, cur_id, resid_slot, s);
    }
}

hipError_t launch_ibm(int storage, const void *prev, void *cur, const DevPtrs &p, int n_cases, int Mtot,
                      int n_mtiles, int maxL3, int cycles, int warm_mode, const _Float16 *th16, int warm_cycles,
                      int diag, int force_surface, int prev_id, hipStream_t s)
{
    if (Mtot == 0) return hipSuccess;
    switch (storage) {
    case ST_MOM:
        return ibm_impl<CodecMom>(prev, cur, p, n_cases, Mtot, n_mtiles, maxL3, cycles, warm_mode, th16, warm_cycles,
                                  diag, force_surface, prev_id, s);
    case ST_F16:
        return ibm_impl<CodecF16>(prev, cur, p, n_cases, Mtot, n_mtiles, maxL3, cycles, warm_mode, th16, warm_cycles,
                                  diag, force_surface, prev_id, s);
    case ST_BF16:
        return ibm_impl<CodecBF16>(prev, cur, p, n_cases, Mtot, n_mtiles, maxL3, cycles, warm_mode, th16,
                                   warm_cycles, diag, force_surface, prev_id, s);
    default:
        return ibm_impl<CodecF32>(prev, cur, p, n_cases, Mtot, n_mtiles, maxL3, cycles, warm_mode, th16, warm_cycles,
                                  diag, force_surface, prev_id, s);
    }
}

hipError_t launch_targets(const DevPtrs &p, int Mtot, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_targets, dim3((Mtot + 255) / 256), dim3(256), 0, s, p, Mtot, out);
    return hipGetLastError();
}

template <class CD>
static hipError_t window_impl(void *cur, const DevPtrs &p, int n_cases, int max_slab, int cur_id, int advance,
                              hipStream_t s)
{
    if (advance)
        hipLaunchKernelGGL(k_window_advance, dim3((n_cases + 63) / 64), dim3(64), 0, s, p, n_cases);
    else
        hipLaunchKernelGGL(k_window_trigger, dim3((n_cases + 63) / 64), dim3(64), 0, s, p, n_cases);
    if (max_slab > 0) {
        // about 2048 workgroups in all, at least 8 per case
        const int per_case = std::max(8, std::min((max_slab + 255) / 256, 2048 / n_cases));
        hipLaunchKernelGGL(k_window_reset<CD>, dim3(per_case, n_cases), dim3(256), 0, s, (typename CD::T *)cur, p,
                           cur_id);
    }
    return hipGetLastError();
}

hipError_t launch_window(int storage, void *cur, const DevPtrs &p, int n_cases, int max_slab, int cur_id, int advance,
                         hipStream_t s)
{
    switch (storage) {
    case ST_MOM: return window_impl<CodecMom>(cur, p, n_cases, max_slab, cur_id, advance, s);
    case ST_F16: return window_impl<CodecF16>(cur, p, n_cases, max_slab, cur_id, advance, s);
    case ST_BF16: return window_impl<CodecBF16>(cur, p, n_cases, max_slab, cur_id, advance, s);
    default: return window_impl<CodecF32>(cur, p, n_cases, max_slab, cur_id, advance, s);
    }
}

}  // namespace turret
