// The integrator half of the fused MD step, shared by every step kernel:
// the final half kick of the previous step with the forces just gathered,
// then B A O A into pos_out (BAOAB, Leimkuhler & Matthews 2013), the path
// length of the skin test, and the per-block status slots.  pos_out receives
// the new positions (a.pos_out, or a workgroup's LDS copy); blk is the logical
// 64-particle block, which names the status slot and the energy row.
#pragma once

#include "rc_gather.h"

namespace rc {

template <bool EV>
__device__ __forceinline__ void step_finish(const StepArgs& a, float4* pos_out, int m, int blk, bool live,
                                            const float4& pm,
                                            const float4& vm, const Acc& acc, const Box& box, int tag0,
                                            uint64_t seed, uint64_t step) {
    float kin[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float path = 0.0f, path_in = 0.0f;
    bool bad = false, lost = false;
    if (live) {
        path_in = vm.w;
        const int tm = ptype(pm.w);
        const float minv = a.minv[tm];
        const float hdt = 0.5f * a.dt;
        float vx = vm.x, vy = vm.y, vz = vm.z;
        if (a.mode == RC_STEP_CONT || a.mode == RC_STEP_FINISH) {  // final B of the previous step
            vx += hdt * acc.fx * minv;
            vy += hdt * acc.fy * minv;
            vz += hdt * acc.fz * minv;
        }
        if (EV) {
            const float mm = 1.0f / minv;
            kin[0] = mm * vx * vx; kin[1] = mm * vy * vy; kin[2] = mm * vz * vz;
            kin[3] = mm * vx * vy; kin[4] = mm * vx * vz; kin[5] = mm * vy * vz;
        }
        if (a.mode == RC_STEP_FINISH || a.mode == RC_STEP_OBSERVE) {
            if (a.mode == RC_STEP_FINISH) a.vel[m] = make_float4(vx, vy, vz, vm.w);
            path = vm.w;
        } else {
            vx += hdt * acc.fx * minv;  // B
            vy += hdt * acc.fy * minv;
            vz += hdt * acc.fz * minv;
            float sx = hdt * vx, sy = hdt * vy, sz = hdt * vz;  // A (first half of the drift)
            if (a.langevin) {                                  // O
                float z0, z1, z2;
                thermostat_normals(seed, (uint32_t)(ptag(pm.w) - tag0), step, z0, z1, z2);
                const float c2 = a.c2[tm];
                vx = a.c1 * vx + c2 * z0;
                vy = a.c1 * vy + c2 * z1;
                vz = a.c1 * vz + c2 * a.noise_z * z2;  // no z noise in the xy plane
            }
            sx += hdt * vx;  // A
            sy += hdt * vy;
            sz += hdt * vz;
            float x = pm.x + sx, y = pm.y + sy, z = pm.z + sz;
            int ix = 0, iy = 0, iz = 0;
            if (x >= box.hf[0]) { x -= box.Lf[0]; ix = 1; } else if (x < -box.hf[0]) { x += box.Lf[0]; ix = -1; }
            if (y >= box.hf[1]) { y -= box.Lf[1]; iy = 1; } else if (y < -box.hf[1]) { y += box.Lf[1]; iy = -1; }
            if (z >= box.hf[2]) { z -= box.Lf[2]; iz = 1; } else if (z < -box.hf[2]) { z += box.Lf[2]; iz = -1; }
            // the path length only gates list builds: the hardware square root (~1 ulp) suffices
            path = vm.w + __builtin_amdgcn_sqrtf(sx * sx + sy * sy + sz * sz);
            lost = fabsf(sx) > box.hf[0] || fabsf(sy) > box.hf[1] || fabsf(sz) > box.hf[2];
            bad = !(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(vx) && isfinite(vy) &&
                    isfinite(vz));
            pos_out[m] = make_float4(x, y, z, pm.w);
            a.vel[m] = make_float4(vx, vy, vz, path);
            if (a.image && (ix | iy | iz)) {
                int4 im = a.image[m];
                im.x += ix;
                im.y += iy;
                im.z += iz;
                a.image[m] = im;
            }
        }
    }
    // ---- status: per-block slots, plain stores (no same-address atomics) ----------
    // Each block (one wave) ORs its flags and keeps its first soft/hard step in
    // its own slot of blk[]; k_fold_status folds the slots once per chunk.
    const bool soft = live && (a.mode == RC_STEP_START || a.mode == RC_STEP_CONT) && path > a.soft;
    const bool hard = live && path_in > a.hard;
    const unsigned long long bs = __ballot(soft), bh = __ballot(hard), bb = __ballot(bad),
                             bl = __ballot(lost);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const int fl = (bs ? RC_FLAG_REBUILD : 0) | (bh ? RC_FLAG_STALE : 0) | (bb ? RC_FLAG_NONFINITE : 0) |
                       (bl ? RC_FLAG_LOST : 0);
        if (fl) {
            int* slot = a.blk + 3 * blk;
            const int st = (int)(step & 0x7fffffff);
            slot[0] |= fl;
            if (fl & RC_FLAG_REBUILD) slot[1] = min(slot[1], st);
            if (fl & RC_FLAG_STALE) slot[2] = min(slot[2], st);
        }
    }
    if (EV) {
        double v[13] = {acc.e,  acc.w[0], acc.w[1], acc.w[2], acc.w[3], acc.w[4], acc.w[5],
                        kin[0], kin[1],   kin[2],   kin[3],   kin[4],   kin[5]};
        wave_sum_store<13>(v, a.ev_part + (size_t)blk * kEvWords);
        if (a.bond_part) {   // the bond count of the positions the forces were gathered at
            unsigned nb = acc.nbond;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) nb += __shfl_xor(nb, o, kWave);
            if ((threadIdx.x & (kWave - 1)) == 0) a.bond_part[blk] = nb;
        }
    }
}

}  // namespace rc
