// Rigid planar bodies for the patchy colloids of Sec. 3.2: a disk (the body's
// centre particle) carrying massless patch particles at fixed body-frame
// offsets.  The forces on every particle come from the stand-alone force
// kernel; this file sums them per body into a force and a torque, advances
// the body's (x, y, angle) by the BAOAB half steps of the particle integrator
// (with the angle driven by the torque, the body's moment of inertia and a
// rotational friction equal to the translational one), and places the patches
// at the new pose.  One thread per body; members are found by tag (rtag).
#include <cmath>

#include "rc_host.h"

namespace rc {

struct RigidArgs {
    float4* pos;
    float4* vel;
    const float4* force;
    int4* image;            // NULL ok
    const int* rtag;
    const int* centre;      // [B] tag of each body's centre particle
    const int* first;       // [B + 1] member range of each body
    const int* member;      // [M] member tags
    const float* offset;    // [M][2] body-frame offsets
    const float* inertia;   // [B]
    float* theta;           // [B] angle in [-pi, pi)
    float* omega;           // [B] angular velocity
    int* status;            // NULL ok
    int B;
    Box box;
    float minv[RC_MAX_TYPES];
    float c2[RC_MAX_TYPES];
    float dt, c1, kT;
    int langevin;
    uint64_t seed, step;
    int half;
};

// minimum image of a separation in the plane (FP32; members lie well within half a box of their centre)
__device__ __forceinline__ float mi(float d, float L, float h) {
    if (d >= h) d -= L;
    else if (d < -h) d += L;
    return d;
}

__device__ __forceinline__ float wrap_coord(float x, float L, float h, int& im) {
    if (x >= h) {
        x -= L;
        ++im;
    } else if (x < -h) {
        x += L;
        --im;
    }
    return x;
}

__global__ __launch_bounds__(kBlock) void k_rigid(RigidArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const Box& bx = a.box;
    const int c = a.rtag[a.centre[b]];
    const float4 pc = a.pos[c];
    const float4 vc = a.vel[c];
    const float minv = a.minv[ptype(pc.w)];
    const float inv_i = 1.0f / a.inertia[b];
    const int m0 = a.first[b], m1 = a.first[b + 1];
    // force and torque (about the centre) of the body
    float fx = a.force[c].x, fy = a.force[c].y, tau = 0.0f;
    for (int m = m0; m < m1; ++m) {
        const int j = a.rtag[a.member[m]];
        const float4 pm = a.pos[j];
        const float4 fm = a.force[j];
        const float dx = mi(pm.x - pc.x, bx.Lf[0], bx.hf[0]), dy = mi(pm.y - pc.y, bx.Lf[1], bx.hf[1]);
        fx += fm.x;
        fy += fm.y;
        tau += dx * fm.y - dy * fm.x;
    }
    const float hdt = 0.5f * a.dt;
    float vx = vc.x + hdt * fx * minv, vy = vc.y + hdt * fy * minv;  // B
    float w = a.omega[b] + hdt * tau * inv_i;
    float th = a.theta[b];
    float x = pc.x, y = pc.y, path = vc.w;
    if (a.half == RC_HALF_FIRST) {
        float sx = hdt * vx, sy = hdt * vy, st = hdt * w;  // A
        if (a.langevin) {                                   // O: the centre's z normal drives the angle
            float z0, z1, z2;
            thermostat_normals(a.seed, (uint32_t)ptag(pc.w), a.step, z0, z1, z2);
            const float c2 = a.c2[ptype(pc.w)];
            vx = a.c1 * vx + c2 * z0;
            vy = a.c1 * vy + c2 * z1;
            w = a.c1 * w + sqrtf((1.0f - a.c1 * a.c1) * a.kT * inv_i) * z2;
        }
        sx += hdt * vx;  // A
        sy += hdt * vy;
        st += hdt * w;
        int ix = 0, iy = 0;
        x = wrap_coord(pc.x + sx, bx.Lf[0], bx.hf[0], ix);
        y = wrap_coord(pc.y + sy, bx.Lf[1], bx.hf[1], iy);
        path += sqrtf(sx * sx + sy * sy);
        th += st;
        const float pi = 3.14159265358979f;
        if (th >= pi) th -= 2.0f * pi;
        else if (th < -pi) th += 2.0f * pi;
        a.pos[c] = make_float4(x, y, pc.z, pc.w);
        if (a.image && (ix | iy)) {
            int4 im = a.image[c];
            im.x += ix;
            im.y += iy;
            a.image[c] = im;
        }
        a.theta[b] = th;
        const bool bad = !(isfinite(x) && isfinite(y) && isfinite(vx) && isfinite(vy) && isfinite(w));
        if (bad && a.status) atomicOr(&a.status[RC_ST_FLAGS], RC_FLAG_NONFINITE);
    }
    a.vel[c] = make_float4(vx, vy, 0.0f, path);
    a.omega[b] = w;
    // members: placed at the pose (first half), velocities v + w x d (both halves)
    float sn, cs;
    sincosf(th, &sn, &cs);
    for (int m = m0; m < m1; ++m) {
        const int j = a.rtag[a.member[m]];
        const float ox = a.offset[2 * m], oy = a.offset[2 * m + 1];
        const float dx = cs * ox - sn * oy, dy = sn * ox + cs * oy;
        const float4 pm = a.pos[j];
        float pmw = a.vel[j].w;
        if (a.half == RC_HALF_FIRST) {
            int ix = 0, iy = 0;
            const float xm = wrap_coord(x + dx, bx.Lf[0], bx.hf[0], ix);
            const float ym = wrap_coord(y + dy, bx.Lf[1], bx.hf[1], iy);
            const float ex = mi(xm - pm.x, bx.Lf[0], bx.hf[0]), ey = mi(ym - pm.y, bx.Lf[1], bx.hf[1]);
            pmw += sqrtf(ex * ex + ey * ey);
            a.pos[j] = make_float4(xm, ym, pm.z, pm.w);
            if (a.image) {  // a member's image follows its own crossings
                const int mx = (xm - pm.x > bx.hf[0]) ? -1 : ((xm - pm.x < -bx.hf[0]) ? 1 : 0);
                const int my = (ym - pm.y > bx.hf[1]) ? -1 : ((ym - pm.y < -bx.hf[1]) ? 1 : 0);
                if (mx | my) {
                    int4 im = a.image[j];
                    im.x += mx;
                    im.y += my;
                    a.image[j] = im;
                }
            }
        }
        a.vel[j] = make_float4(vx - w * dy, vy + w * dx, 0.0f, pmw);
    }
}

}  // namespace rc

using namespace rc;
using namespace rc::host;

extern "C" int rc_rigid_step(rc_ctx* c, float* pos, float* vel, const float* force, int* image, const int* rtag,
                             int B, const int* centre, const int* first, const int* member, const float* offset,
                             const float* inertia, float* theta, float* omega, int N, rc_box box,
                             const rc_integrator* cfg, uint64_t step, int half, int* status, void* stream) {
    if (c) c->md.valid = false;   // the state changes outside the driver
    if (!c) return RC_ERR_ARG;
    if (N < 1 || B < 1 || B > N) return fail(c, RC_ERR_ARG, "need 1 <= B <= N (B = %d, N = %d)", B, N);
    if (!pos || !vel || !force || !rtag || !centre || !first || !member || !offset || !inertia || !theta ||
        !omega)
        return fail(c, RC_ERR_ARG, "rc_rigid_step: a required array is NULL");
    if (half != RC_HALF_FIRST && half != RC_HALF_SECOND) return fail(c, RC_ERR_ARG, "half must be 0 or 1");
    if (!cfg || cfg->dim != 2) return fail(c, RC_ERR_ARG, "rigid planar bodies need an integrator of dim 2");
    RigidArgs a{};
    int lang = 0;
    float nz = 0.0f;
    int r = check_integrator(c, cfg, a.minv, a.c2, a.c1, lang, nz);
    if (r) return r;
    if ((r = make_box(c, box, a.box))) return r;
    a.pos = reinterpret_cast<float4*>(pos);
    a.vel = reinterpret_cast<float4*>(vel);
    a.force = reinterpret_cast<const float4*>(force);
    a.image = reinterpret_cast<int4*>(image);
    a.rtag = rtag;
    a.centre = centre;
    a.first = first;
    a.member = member;
    a.offset = offset;
    a.inertia = inertia;
    a.theta = theta;
    a.omega = omega;
    a.status = status;
    a.B = B;
    a.dt = (float)cfg->dt;
    a.kT = (float)cfg->kT;
    a.langevin = lang;
    a.seed = cfg->seed;
    a.step = step;
    a.half = half;
    hipLaunchKernelGGL(k_rigid, dim3(nblocks(B, kBlock)), dim3(kBlock), 0, S(stream), a);
    HIP_TRY(c, hipGetLastError());
    return RC_OK;
}
