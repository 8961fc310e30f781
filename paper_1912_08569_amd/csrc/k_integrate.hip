// Standalone BAOAB / velocity-Verlet half steps (rc_integrate_step).
#include <algorithm>
#include "rc_internal.h"

namespace rc {

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

template <bool KIN>
__global__ __launch_bounds__(kBlock) void k_integrate(IntegrateArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < a.N;
    float kin[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    bool soft = false, bad = false, lost = false;
    if (live) {
        const float4 p = a.pos[i];
        const float4 v = a.vel[i];
        const float4 f = a.force[i];
        const int t = ptype(p.w);
        const float minv = a.minv[t], hdt = 0.5f * a.dt;
        float vx = v.x + hdt * f.x * minv, vy = v.y + hdt * f.y * minv, vz = v.z + hdt * f.z * minv;
        float path = v.w;
        if (a.half == RC_HALF_FIRST) {
            float sx = hdt * vx, sy = hdt * vy, sz = hdt * vz;
            if (a.langevin) {
                float z0, z1, z2;
                thermostat_normals(a.seed, (uint32_t)ptag(p.w), a.step, z0, z1, z2);
                const float c2 = a.c2[t];
                vx = a.c1 * vx + c2 * z0;
                vy = a.c1 * vy + c2 * z1;
                vz = a.c1 * vz + c2 * a.noise_z * z2;  // no z noise in the xy plane
            }
            sx += hdt * vx;
            sy += hdt * vy;
            sz += hdt * vz;
            float x = p.x + sx, y = p.y + sy, z = p.z + sz;
            int ix = 0, iy = 0, iz = 0;
            if (x >= a.box.hf[0]) { x -= a.box.Lf[0]; ix = 1; } else if (x < -a.box.hf[0]) { x += a.box.Lf[0]; ix = -1; }
            if (y >= a.box.hf[1]) { y -= a.box.Lf[1]; iy = 1; } else if (y < -a.box.hf[1]) { y += a.box.Lf[1]; iy = -1; }
            if (z >= a.box.hf[2]) { z -= a.box.Lf[2]; iz = 1; } else if (z < -a.box.hf[2]) { z += a.box.Lf[2]; iz = -1; }
            path += __builtin_amdgcn_sqrtf(sx * sx + sy * sy + sz * sz);  // as the fused step
            lost = fabsf(sx) > a.box.hf[0] || fabsf(sy) > a.box.hf[1] || fabsf(sz) > a.box.hf[2];
            bad = !(isfinite(x) && isfinite(y) && isfinite(z));
            soft = path > a.soft;
            a.pos[i] = make_float4(x, y, z, p.w);
            if (a.image && (ix | iy | iz)) {
                int4 im = a.image[i];
                im.x += ix;
                im.y += iy;
                im.z += iz;
                a.image[i] = im;
            }
        }
        bad = bad || !(isfinite(vx) && isfinite(vy) && isfinite(vz));
        a.vel[i] = make_float4(vx, vy, vz, path);
        if (KIN) {
            const float m = 1.0f / minv;
            kin[0] = m * vx * vx; kin[1] = m * vy * vy; kin[2] = m * vz * vz;
            kin[3] = m * vx * vy; kin[4] = m * vx * vz; kin[5] = m * vy * vz;
        }
    }
    if (a.status) {
        const unsigned long long bs = __ballot(soft), bb = __ballot(bad), bl = __ballot(lost);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            int fl = (bs ? RC_FLAG_REBUILD : 0) | (bb ? RC_FLAG_NONFINITE : 0) | (bl ? RC_FLAG_LOST : 0);
            if (fl) atomicOr(&a.status[RC_ST_FLAGS], fl);
        }
    }
    if (KIN) {
        double v[6] = {kin[0], kin[1], kin[2], kin[3], kin[4], kin[5]};
        block_sum_store<6>(v, a.kin_part + (size_t)blockIdx.x * kEvWords + 7);
    }
}

// The thermostat normals of tags [0, N) at steps step0 .. step0 + steps - 1,
// as every integrating kernel draws them: out[k * N + t] = (xi_x, xi_y, xi_z, 0).
__global__ __launch_bounds__(kBlock) void k_thermostat_normals(uint64_t seed, uint64_t step0, int steps, int N,
                                                              float noise_z, float4* __restrict__ out) {
    const long total = (long)steps * N;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const long k = i / N;
        const int t = (int)(i - k * N);
        float z0, z1, z2;
        thermostat_normals(seed, (uint32_t)t, step0 + (uint64_t)k, z0, z1, z2);
        out[i] = make_float4(z0, z1, noise_z * z2, 0.0f);
    }
}

hipError_t launch_thermostat_normals(uint64_t seed, uint64_t step0, int steps, int N, float noise_z, float4* out,
                                     hipStream_t s) {
    const long total = (long)steps * N;
    const int blocks = (int)std::min<long>((total + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_thermostat_normals, dim3(blocks), dim3(kBlock), 0, s, seed, step0, steps, N, noise_z, out);
    return hipGetLastError();
}

hipError_t launch_integrate(const IntegrateArgs& a, hipStream_t s) {
    if (a.kin_part)
        hipLaunchKernelGGL(k_integrate<true>, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_integrate<false>, dim3(nblk(a.N, kBlock)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace rc
