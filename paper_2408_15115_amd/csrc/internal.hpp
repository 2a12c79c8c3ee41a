// internal.hpp -- device-side descriptors shared by the kernels and the C-ABI
// layer of libturret (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace turret {

// Static description of one case, in device memory.
struct CaseDev {
    int nx, ny, nz;
    int bc_lo, bc_hi, sponge;
    int M, marker_off;      // markers of this case: [marker_off, marker_off + M)
    int tile_off, n_tiles;  // marker tiles of this case: [tile_off, tile_off + n_tiles)
    int L, dz;              // IBM region edge (cells) and window shift rows
    long long cells;        // nx * ny * nz
    long long plane;        // elements per direction plane (cells rounded up to 128)
    long long pop_off;      // element offset of the case block in the population buffers
    long long reg_off;      // cell offset of the case region in the region pool
    float tau0;
    int forcing;            // 0: forced rule as printed; 1: momentum-exact variant
    double h_ini, h_end;
    double force_offset;    // 0: stress integral at the markers; > 0: on the parallel surface
    float uw_lo, uw_hi;     // x velocity of a no-slip bottom / top wall
    long long xreg_off;     // moment storage: cell offset of the case's expanded region (edge L + 2)
    int LB[3];              // FP16/BF16 storage: edges of the case's full-precision box (0: none)
    long long fine_off;     // element offset of the case's box in each box buffer ([27][LBz][LBy][LBx])
};

// Dynamic FP64 rigid-body state of one case plus the ring origin and region
// origin, in device memory (Sec. 2.3; window of Sec. 2.5).
struct BodyDev {
    double r[3], d[9], v[3], w[3];
    double F[3], T[3], Fp[3];
    double Text[3];  // constant external torque (lab frame)
    double kappa, vol, Jm_inv[9], gravity, Rb, resid;
    int z0;          // ring origin: physical row z is stored in slot (z + z0) mod nz
    int shift_now;   // 1 if the window moved during the last window_shift
    int shifts, steps;
    double gate;                // learned start accepted while its residual is <= gate
    double resid_hist[16];      // per-cycle residuals: [0..7] first sequence, [8..15] fallback
    int accepts, rejects;       // learned-start decisions so far
    int fallback;               // 1 if the last step fell back to the plain start
    int active;                 // 1 while the case still runs cycles of the current sequence
    int dorg[3];                // moment storage: forcing-box origin (x, y, ring slot) of the last correction
    int dvalid;                 // moment storage: 1 once a correction has written the forcing box
    int warm_cyc_sum;           // cycles used by the accepted learned starts, summed
    int org[3];      // IBM region origin (physical cell coordinates, x/y unwrapped)
    int fo[2][3];    // full-precision box origin of population buffer 0 / 1 (physical, x/y unwrapped)
    int fvalid[2];   // 1 once a step has written that buffer's box
    unsigned int logged;          // records written to the case's step log so far
    unsigned int pad_;
    int err;         // 1: a marker stencil left the box in z; 2: non-finite or huge IBM value;
                     // 4: non-finite density or |u| > 0.5.  Nonzero masks (freezes) the case.
};

struct Tile {
    int c;           // case
    int first;       // first cell (flat index inside the case) of the tile
};

// A marker tile: up to kTileMarkers markers of one case that lie close
// together on the body (sorted along a Morton curve of their body-frame
// positions, at most kTileSpan lattice units apart per axis), handled by one
// workgroup whose stencils share a box of at most kBoxCells cells staged in
// LDS.
struct MarkerTile {
    int c, first, count, pad;
};
// Box of region cells covering the stencils of a tile's markers.
struct TileBox {
    int lo[3];    // first stencil node of the box (physical cell coordinates, x/y unwrapped)
    int o[3];     // the same as region coordinates
    int e[3];     // box extent
    int fits;     // 1 if the box has at most kBoxCells cells and lies inside the region
};
constexpr int kTileMarkers = 16;
constexpr double kTileSpan = 3.0;
// LDS box capacity: a tile spans at most kTileSpan per axis in the body frame,
// so its box is at most 7^3 cells axis-aligned and stays at or below 448
// cells in the rotations measured (random orientations of the 12k-marker
// ellipsoid); larger boxes take the per-node HBM path.  448 keeps the force
// kernel (10 FP32 fields + 3 int64 accumulators per cell, plus the markers'
// records) under 32 KB of LDS, five workgroups per CU.
constexpr int kBoxCells = 448;

// Fixed-point scale of the deterministic immersed-force accumulator.
constexpr double kFixScale = 1099511627776.0;   // 2^40
constexpr double kFixInv = 1.0 / 1099511627776.0;
// Immersed-force accumulators: the spread of forcing cycle c goes to
// accumulator c - 1, so that one kernel can interpolate cycle c (reading
// accumulators 0 .. c-1) and spread cycle c + 1 without a race; their sum is
// the immersed force H.  Paths with more cycles use accumulator 0 alone.
constexpr int kHBufs = 4;

// Per-tile partial sums written by the force kernels: F(3) T(3) Fp(3).
constexpr int kPart = 9;
// Region fields: rho - 1, u (3), sigma xx yy zz xy xz yz (6).
constexpr int kRegFields = 10;

struct DevPtrs {
    CaseDev *cases;
    BodyDev *body;
    Tile *tiles;
    int *mcase;
    double *xb, *nb, *dS;
    double *X, *N, *U, *hk, *dh;
    double *part;    // per-tile force, torque and pressure-force sums (kPart each)
    double *res;     // per-tile max residual of the last interpolation
    double *wt;      // per-marker one-dimensional stencil weights, w[4 d + o] for node floor(X_d) - 1 + o
    unsigned char *mark;   // per region cell: 1 if inside a tile's stencil box this step
    float *reg;
    long long *H;    // kHBufs fixed-point immersed-force accumulators, hstride elements apart
    long long hstride;
    int *counter;    // 8 work-queue counters of the persistent lattice schedule
    MarkerTile *mtiles;
    float *feat;     // per-marker warm-start features (12)
    double *h0;      // per-marker plain start U - I[u*] (3)
    double *hk2;     // per-marker final h of the step before the previous one (3)
    double *hs;      // per-marker scale of the warm-start features, |h0| + |h(t-1)|
    double *dSo;     // per-marker areas of the parallel force surface (cases with force_offset > 0)
    TileBox *tbox;   // per-tile boxes of the markers' stencils, then of the force-surface points', by k_markers
    float *dsh;      // moment storage: per region cell the forcing shift (Delta_x, Delta_y, Delta_z, lambda)
    float *rpop;     // moment storage: collided populations of the region and a one-cell rim, [27][xstride]
    long long xstride;
    float *fine[2];  // FP16/BF16 storage: the full-precision boxes of population buffers 0 and 1
    double *log;     // per case a ring of kLogCap step records of kLogFields values
};

// Step log: at the end of every step each case appends one record, in the
// layout of the body-state read (r, d, v, w, F, T, F_pressure, residual,
// steps, shifts, z0, err), to a ring of kLogCap records.
constexpr int kLogCap = 1024;
constexpr int kLogFields = 32;

// ---------------------------------------------------------------- launchers
// collision: 0 = recursive regularized, 1 = BGK (comparison; plain schedule)
hipError_t launch_stream_collide(int storage, const void *src, void *dst, const DevPtrs &p, int ntiles,
                                 int block, int schedule, int persist_wgs, int collision, hipStream_t s);
// The D3Q19 comparison lattice (fluid only, FP32, periodic, plain schedule).
hipError_t launch_stream_collide19(const void *src, void *dst, const DevPtrs &p, int ntiles, int block,
                                   int collision, hipStream_t s);
// Moment storage (FP32): the z-marching step over the moment tile table, and
// per-case conversions between moments (with the forcing shifts of the last
// correction) and population deviations ([10][plane] <-> [27][plane]).
int moment_tiles(int nx, int ny, int nz);
hipError_t launch_moment_step(const void *src, void *dst, const DevPtrs &p, int ntiles, hipStream_t s);
hipError_t launch_moments_expand(const float *src, float *dst, const DevPtrs &p, int c, hipStream_t s);
// the same with the case's cell count from the host plan (no synchronizing read)
hipError_t launch_moments_expand_n(const float *src, float *dst, const DevPtrs &p, int c, long long cells,
                                   hipStream_t s);
hipError_t launch_moments_project(const float *src, float *dst, long long plane, long long cells, hipStream_t s);
hipError_t launch_body_advance(const DevPtrs &p, int n_cases, hipStream_t s);
// FP16/BF16 storage with full-precision boxes: after the lattice kernel,
// step the box cells again from buffer sid's box into buffer did's box
// (max_box = the largest box's cell count; 0 = no boxes).
hipError_t launch_fine_step(int storage, const void *src, void *dst, const DevPtrs &p, int sid, int did, int n_cases,
                            long long max_box, int collision, hipStream_t s);
// IBM coupling.  With a warm start (warm_mode 1: the previous step's final
// h_k; 2: the network th16) cycles run from that start until a case's
// residual is at or below its gate, at most warm_cycles of them; cases that
// do not get there rerun `cycles` plain cycles.  diag keeps the residual of
// every cycle.
// force_surface: some case evaluates the force on its parallel surface.
// launch_ibm runs the coupling up to h(t+1) (it reads `prev`, the buffer the
// lattice kernel reads, not the lattice kernel's output, so it may run
// beside it); launch_correct then adds the forcing to `cur`.
// prev_id / cur_id: the population buffer (0 or 1) of prev / cur, whose
// full-precision box the kernels read / update.
hipError_t launch_ibm(int storage, const void *prev, void *cur, const DevPtrs &p, int n_cases, int Mtot,
                      int n_mtiles, int maxL3, int cycles, int warm_mode, const _Float16 *th16, int warm_cycles,
                      int diag, int force_surface, int prev_id, hipStream_t s);
// resid_slot >= 0: the correction also forms the case residual of the plain
// fused forcing sequence (whose last pass leaves the tile maxima) into
// resid and resid_hist[resid_slot].
hipError_t launch_correct(int storage, void *cur, const DevPtrs &p, int n_cases, int Mtot, int maxL3, int cur_id,
                          int resid_slot, hipStream_t s);
// Whether the plain forcing sequence runs fused (each spread in the preceding
// interpolation pass); it then leaves its residual to the correction.
inline bool ibm_fused(int warm_mode, int cycles) { return warm_mode == 0 && cycles <= kHBufs; }
hipError_t launch_targets(const DevPtrs &p, int Mtot, float *out, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, long long bytes, hipStream_t s);
// The window test and reset of Sec. 2.5; with advance set, the test and the
// next step's body advance run in one kernel (identical results).
hipError_t launch_window(int storage, void *cur, const DevPtrs &p, int n_cases, int max_slab, int cur_id, int advance,
                         hipStream_t s);

}  // namespace turret
