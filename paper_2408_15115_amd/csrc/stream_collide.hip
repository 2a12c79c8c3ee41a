// stream_collide.hip -- the fused pull-streaming + recursive-regularized
// collision kernel of the lattice Boltzmann step (arXiv 2408.15115, Sec. 2.1
// and App. A), one thread per cell over SoA storage, its launch schedules,
// and the plain streaming copy that calibrates HBM bandwidth and counters.
#include <type_traits>

#include "fine.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "pull.hpp"

namespace turret {

// Every population is written once per step and not read again before the
// next step: the stores carry the non-temporal hint (measured faster; the
// same hint on the loads is not).
template <class CD>
__device__ __forceinline__ void store_all(typename CD::T *__restrict__ dst, long long plane, int off, const float out[Q])
{
    Unroll<0, Q>::run([&](auto I) {
        constexpr int i = decltype(I)::value;
        __builtin_nontemporal_store(CD::template enc<i>(out[i]), &dst[(long long)i * plane + off]);
    });
}

// ------------------------------------------------------------ stream-collide
// One tile = blockDim.x consecutive cells of one case.  A case whose error
// bits are set is masked (frozen) so the rest of a batch goes on.  The guard
// flags non-finite density or |u| > 0.5 (bit 4) with one atomic per wave.
// COLL 0: recursive-regularized collision (App. A); COLL 1: BGK for
// comparison, f0 + (1 - 1/tau)(f - f0) with the raw off-equilibrium.
template <class CD, int COLL>
__device__ __forceinline__ void stream_collide_tile(const typename CD::T *__restrict__ src, typename CD::T *__restrict__ dst,
                                                    const CaseDev *__restrict__ cases, BodyDev *__restrict__ body, Tile tl,
                                                    int off)
{
    const CaseDev &cd = cases[tl.c];
    const int nx = cd.nx, ny = cd.ny, nz = cd.nz;
    const int cell = tl.first + off;   // off: this thread's cell in the tile
    if (body[tl.c].err != 0 || cell >= (int)cd.cells) return;
    const int z0 = body[tl.c].z0;
    const int x = cell % nx;
    const int t2 = cell / nx;
    const int y = t2 % ny;
    const int z = t2 / ny;
    // FP16 / BF16 with the full-precision box: the box step writes the box's
    // cells (it may run beside this kernel), so their stores are skipped
    // here (the cells are still collided for the stability guard).  The box
    // of this step starts one cell before the particle region, whose origin
    // the body advance has set.
    bool in_box = false;
    if constexpr (!std::is_same<CD, CodecF32>::value) {
        if (cd.LB[0] > 0) {
            const BodyDev &Bb = body[tl.c];
            int kx = x - wrap_mod(Bb.org[0] - 1, nx), ky = y - wrap_mod(Bb.org[1] - 1, ny);
            kx += kx < 0 ? nx : 0;
            ky += ky < 0 ? ny : 0;
            const int kz = z - (Bb.org[2] - 1);
            in_box = kx < cd.LB[0] && ky < cd.LB[1] && kz >= 0 && kz < cd.LB[2];
        }
    }
    float g[Q];
    pull<CD>(src + cd.pop_off, cd.plane, nx, ny, nz, z0, cd.bc_lo, cd.bc_hi, cd.uw_lo, cd.uw_hi, x, y, z, g);
    const Macro M = macro(raw_moments(g));
    const float u2 = M.u[0] * M.u[0] + M.u[1] * M.u[1] + M.u[2] * M.u[2];
    const bool bad = !(fabsf(M.r1) < 1.0f) || !(u2 < 0.25f);
    const unsigned long long m = __ballot(bad);
    if (m != 0ull && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) atomicOr(&body[tl.c].err, 4);
    const float tau = tau_at(cd.tau0, nz, cd.sponge, z);
    const float om = 1.0f - 1.0f / tau;
    float A[Q], out[Q];
    if constexpr (COLL == 1) {
        post_collision_coeffs(M, M.u, 0.0f, A);   // equilibrium coefficients only
        hermite_to_populations(A, out);
#pragma unroll
        for (int i = 0; i < Q; i++) out[i] += om * (g[i] - out[i]);
    } else {
        post_collision_coeffs(M, M.u, om, A);
        hermite_to_populations(A, out);
    }
    if (in_box) return;
    int zc = z + z0;
    if (zc >= nz) zc -= nz;
    store_all<CD>(dst + cd.pop_off, cd.plane, (zc * ny + y) * nx + x, out);
}

// SCHED 0: tile = workgroup; 1: XCD-grouped tiles (workgroups go
// round-robin over the 8 XCDs, so workgroup b handles tile
// (b mod 8) * (grid / 8) + b / 8 and neighbouring rows share one L2);
// 2: persistent workgroups striding over the table; 3: persistent work
// queue.  The queue is split in 8 contiguous segments with one counter each
// (a single device-wide counter serializes every grab across the XCDs);
// workgroup b starts on segment b mod 8, takes kQueueChunk tiles per grab and
// moves on to the other segments when its own is exhausted.  Counters only
// grow, so every workgroup leaves the loop.  4: the same 8 counters, but
// interleaved: counter g hands out chunks g, g + 8, g + 16, ... of the whole
// table, so the 8 XCDs advance through the table side by side and only the
// cases around one point of the table stream at a time (with contiguous
// segments each XCD streams a case of its own, 8 times the plane streams).
// (A queue of single wavefronts, without the barriers, was slower: four
// times the grabs on the same counters.)
// One instantiation per schedule keeps the register allocation of the plain
// schedules free of the loops.
constexpr int kQueueChunk = 4;

template <class CD, int SCHED, int COLL = 0>
__global__ void __launch_bounds__(256) k_stream_collide(const typename CD::T *__restrict__ src,
                                                        typename CD::T *__restrict__ dst,
                                                        const CaseDev *__restrict__ cases, BodyDev *__restrict__ body,
                                                        const Tile *__restrict__ tiles, int ntiles,
                                                        int *__restrict__ counter)
{
    if constexpr (SCHED == 3) {
        __shared__ int s_t;
        const int per = (ntiles + 7) >> 3;
        for (int k = 0; k < 8; k++) {
            const int grp = (blockIdx.x + k) & 7;
            const int lo = grp * per, hi = min(ntiles, lo + per);
            for (;;) {
                if (threadIdx.x == 0) s_t = lo + kQueueChunk * atomicAdd(&counter[grp], 1);
                __syncthreads();
                const int t0 = __builtin_amdgcn_readfirstlane(s_t);
                __syncthreads();
                if (t0 >= hi) break;
                const int t1 = min(t0 + kQueueChunk, hi);
                for (int t = t0; t < t1; t++) stream_collide_tile<CD, COLL>(src, dst, cases, body, tiles[t], (int)threadIdx.x);
            }
        }
    } else if constexpr (SCHED == 4) {
        __shared__ int s_j;
        const int nchunks = (ntiles + kQueueChunk - 1) / kQueueChunk;
        for (int k = 0; k < 8; k++) {
            const int grp = (blockIdx.x + k) & 7;
            for (;;) {
                if (threadIdx.x == 0) s_j = atomicAdd(&counter[grp], 1);
                __syncthreads();
                const int chunk = 8 * __builtin_amdgcn_readfirstlane(s_j) + grp;
                __syncthreads();
                if (chunk >= nchunks) break;
                const int t0 = chunk * kQueueChunk, t1 = min(t0 + kQueueChunk, ntiles);
                for (int t = t0; t < t1; t++) stream_collide_tile<CD, COLL>(src, dst, cases, body, tiles[t], (int)threadIdx.x);
            }
        }
    } else if constexpr (SCHED == 2) {
        for (int t = blockIdx.x; t < ntiles; t += gridDim.x) stream_collide_tile<CD, COLL>(src, dst, cases, body, tiles[t], (int)threadIdx.x);
    } else {
        int t = blockIdx.x;
        if constexpr (SCHED == 1) t = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
        if (t < ntiles) stream_collide_tile<CD, COLL>(src, dst, cases, body, tiles[t], (int)threadIdx.x);
    }
}

__global__ void k_reset_counter(int *counter)
{
    if (threadIdx.x < 8) counter[threadIdx.x] = 0;
}

// ------------------------------------------------------------ copy kernel
// Plain copy, one 16-byte element per lane and one element per thread (a
// flat grid reaches a higher HBM rate than a grid-strided loop).
__global__ void __launch_bounds__(256) k_copy(int4 *__restrict__ dst, const int4 *__restrict__ src, long long n)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy(void *dst, const void *src, long long bytes, hipStream_t s)
{
    const long long n = bytes / 16;
    const long long grid = (n + 255) / 256;
    if (grid < 1 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(256), 0, s, (int4 *)dst, (const int4 *)src, n);
    return hipGetLastError();
}

// --------------------------------------------------------------- launchers
template <class CD>
static hipError_t stream_collide_impl(const void *src, void *dst, const DevPtrs &p, int ntiles, int block,
                                      int schedule, int persist_wgs, int collision, hipStream_t s)
{
    using T = typename CD::T;
    if (collision == 1) {   // the comparison collision runs with the plain schedule only
        hipLaunchKernelGGL((k_stream_collide<CD, 0, 1>), dim3(ntiles), dim3(block), 0, s, (const T *)src, (T *)dst,
                           p.cases, p.body, p.tiles, ntiles, p.counter);
        return hipGetLastError();
    }
    int grid = ntiles;
    if (schedule == 1) grid = (ntiles + 7) / 8 * 8;
    if (schedule >= 2) grid = persist_wgs > 0 ? persist_wgs : 2048;
    const T *a = (const T *)src;
    T *b = (T *)dst;
    switch (schedule) {
    case 1:
        hipLaunchKernelGGL((k_stream_collide<CD, 1>), dim3(grid), dim3(block), 0, s, a, b, p.cases, p.body, p.tiles,
                           ntiles, p.counter);
        break;
    case 2:
        hipLaunchKernelGGL((k_stream_collide<CD, 2>), dim3(grid), dim3(block), 0, s, a, b, p.cases, p.body, p.tiles,
                           ntiles, p.counter);
        break;
    case 3:
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, p.counter);
        hipLaunchKernelGGL((k_stream_collide<CD, 3>), dim3(grid), dim3(block), 0, s, a, b, p.cases, p.body, p.tiles,
                           ntiles, p.counter);
        break;
    case 4:
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, p.counter);
        hipLaunchKernelGGL((k_stream_collide<CD, 4>), dim3(grid), dim3(block), 0, s, a, b, p.cases, p.body, p.tiles,
                           ntiles, p.counter);
        break;
    default:
        hipLaunchKernelGGL((k_stream_collide<CD, 0>), dim3(grid), dim3(block), 0, s, a, b, p.cases, p.body, p.tiles,
                           ntiles, p.counter);
    }
    return hipGetLastError();
}

hipError_t launch_stream_collide(int storage, const void *src, void *dst, const DevPtrs &p, int ntiles,
                                 int block, int schedule, int persist_wgs, int collision, hipStream_t s)
{
    switch (storage) {
    case ST_F16:
        return stream_collide_impl<CodecF16>(src, dst, p, ntiles, block, schedule, persist_wgs, collision, s);
    case ST_BF16:
        return stream_collide_impl<CodecBF16>(src, dst, p, ntiles, block, schedule, persist_wgs, collision, s);
    default:
        return stream_collide_impl<CodecF32>(src, dst, p, ntiles, block, schedule, persist_wgs, collision, s);
    }
}

}  // namespace turret
