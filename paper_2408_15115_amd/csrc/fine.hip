// fine.hip -- the full-precision box of the FP16/BF16 storage forms (see
// fine.hpp): after the lattice kernel has stepped every cell from the
// reduced-precision store, the box cells around each body are stepped again
// from FP32 sources wherever those lie in the previous box, with the same
// collision (Sec. 2.1, App. A).  Their FP32 results go to the new box and
// their roundings to the store, over the lattice kernel's values.
#include "fine.hpp"
#include "internal.hpp"
#include "lattice.hpp"

namespace turret {

// Compiled for 8 waves per SIMD (at most 64 VGPRs): it runs beside the
// lattice kernel, whose waves hold 64 VGPRs each, and only fits the slots
// they free with the same budget.
template <class CD, int COLL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) k_fine_step(const typename CD::T *__restrict__ src,
                                                   typename CD::T *__restrict__ dst, DevPtrs p, int sid, int did)
{
    const int c = blockIdx.y;
    const CaseDev cd = p.cases[c];
    BodyDev &Bw = p.body[c];
    if (cd.LB[0] == 0 || Bw.err != 0) return;
    // the new box: the particle region of this step (its origin set by the
    // body advance) and a one-cell rim
    const int fo_d[3] = {Bw.org[0] - 1, Bw.org[1] - 1, Bw.org[2] - 1};
    const int fo_s[3] = {Bw.fo[sid][0], Bw.fo[sid][1], Bw.fo[sid][2]};
    const int valid = Bw.fvalid[sid];
    const int z0 = Bw.z0;
    const long long fplane = fine_plane(cd);
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q == 0) {
#pragma unroll
        for (int a = 0; a < 3; a++) Bw.fo[did][a] = fo_d[a];
        Bw.fvalid[did] = 1;
    }
    if (q >= fplane) return;
    const int kx = (int)(q % cd.LB[0]), ky = (int)((q / cd.LB[0]) % cd.LB[1]), kz = (int)(q / (cd.LB[0] * cd.LB[1]));
    const int z = fo_d[2] + kz;
    if (z < 0 || z >= cd.nz) return;
    const int x = wrap_mod(fo_d[0] + kx, cd.nx), y = wrap_mod(fo_d[1] + ky, cd.ny);
    float g[Q];
    pull_fine<CD>(src + cd.pop_off, valid ? p.fine[sid] + cd.fine_off : nullptr, cd, z0, fo_s, x, y, z, g);
    const Macro M = macro(raw_moments(g));
    const float tau = tau_at(cd.tau0, cd.nz, cd.sponge, z);
    const float om = 1.0f - 1.0f / tau;
    float A[Q], out[Q];
    if constexpr (COLL == 1) {
        post_collision_coeffs(M, M.u, 0.0f, A);
        hermite_to_populations(A, out);
#pragma unroll
        for (int i = 0; i < Q; i++) out[i] += om * (g[i] - out[i]);
    } else {
        post_collision_coeffs(M, M.u, om, A);
        hermite_to_populations(A, out);
    }
    int zc = z + z0;
    if (zc >= cd.nz) zc -= cd.nz;
    const long long off = (long long)(zc * cd.ny + y) * cd.nx + x;
    float *F = p.fine[did] + cd.fine_off;
    typename CD::T *D = dst + cd.pop_off;
    Unroll<0, Q>::run([&](auto I) {
        constexpr int i = decltype(I)::value;
        F[(long long)i * fplane + q] = out[i];
        D[(long long)i * cd.plane + off] = CD::template enc<i>(out[i]);
    });
}

template <class CD>
static hipError_t fine_impl(const void *src, void *dst, const DevPtrs &p, int sid, int did, int n_cases,
                            long long max_box, int collision, hipStream_t s)
{
    using T = typename CD::T;
    const dim3 grid((unsigned)((max_box + 255) / 256), n_cases);
    if (collision == 1)
        hipLaunchKernelGGL((k_fine_step<CD, 1>), grid, dim3(256), 0, s, (const T *)src, (T *)dst, p, sid, did);
    else
        hipLaunchKernelGGL((k_fine_step<CD, 0>), grid, dim3(256), 0, s, (const T *)src, (T *)dst, p, sid, did);
    return hipGetLastError();
}

hipError_t launch_fine_step(int storage, const void *src, void *dst, const DevPtrs &p, int sid, int did, int n_cases,
                            long long max_box, int collision, hipStream_t s)
{
    if (max_box <= 0) return hipSuccess;
    switch (storage) {
    case ST_F16: return fine_impl<CodecF16>(src, dst, p, sid, did, n_cases, max_box, collision, s);
    case ST_BF16: return fine_impl<CodecBF16>(src, dst, p, sid, did, n_cases, max_box, collision, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace turret
