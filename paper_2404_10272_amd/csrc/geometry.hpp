// Device-side binary32 ray/grid geometry shared by the sampler kernels.
//
// Every value that decides which voxel owns a ray parameter, or which
// lattice point is a sample, is computed with one IEEE round-to-nearest
// operation at a time and no contraction into fused multiply-add:
//   h = fl((A-B)/R), P(m) = fl(B + fl(m*h)), r = fl(1/d),
//   T(m) = fl(fl(P(m) - o) * r).
// Cheap estimates (floor of the hit position) only pick a starting index;
// exact comparisons against T(m) then settle it, so the result is the
// ownership rule itself: a voxel owns (entry, exit] of the ray parameter.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ogv {

// One axis of one cascade level as seen by one ray, in "ray order": plane
// k = 0..R is met at nondecreasing parameter Tk(k); voxel u lies between
// planes u and u+1.  For d > 0 ray order is index order (m = k); for d < 0
// it is reversed (m = R - k, voxel index R-1-u).
struct Axis {
    float B, h;   // plane m at fl(B + fl(m*h))
    float o, d, r;  // origin and direction component, r = fl(1/d)
    float inv_h;  // approximate 1/h, for index estimates only
    int32_t R;
    bool pos;     // d > 0
    bool zero;    // d == 0 or 1/d infinite: the coordinate never changes

    __device__ __forceinline__ float plane(int m) const {
        float mh = __fmul_rn((float)m, h);
        return __fadd_rn(B, mh);
    }
    // crossing parameter of the plane with ray-order index k
    __device__ __forceinline__ float Tk(int k) const {
        int m = pos ? k : R - k;
        return __fmul_rn(__fsub_rn(plane(m), o), r);
    }
    // voxel index of ray-order voxel u
    __device__ __forceinline__ int voxel(int u) const { return pos ? u : R - 1 - u; }

    // Ray-order voxel owning t (inclusive = false) or the parameters just
    // after t (inclusive = true): the largest k with Tk(k) < t (resp. <=),
    // or -1.  Result in [-1, R].
    __device__ __forceinline__ int locate(float t, bool inclusive) const {
        // estimate from the hit position; any value works, it is corrected
        float p = o + t * d;
        float vf = floorf((p - B) * inv_h);
        float uf = pos ? vf : (float)(R - 1) - vf;
        uf = fminf(fmaxf(uf, -1.0f), (float)R);   // NaN -> -1
        int u = (int)uf;
        if (inclusive) {
            while (u >= 0 && !(Tk(u) <= t)) --u;
            while (u < R && Tk(u + 1) <= t) ++u;
        } else {
            while (u >= 0 && !(Tk(u) < t)) --u;
            while (u < R && Tk(u + 1) < t) ++u;
        }
        return u;
    }

    // Voxel index holding o for a zero axis (floor rule): the v with
    // P(v) <= o < P(v+1); -1 below the grid, R above it.
    __device__ __forceinline__ int zero_voxel() const {
        float vf = floorf((o - B) * inv_h);
        vf = fminf(fmaxf(vf, -1.0f), (float)R);
        int v = (int)vf;
        while (v >= 0 && plane(v) > o) --v;
        while (v < R && plane(v + 1) <= o) ++v;
        return v;
    }

    // Advance ray-order voxel u (known to satisfy Tk(u) <= t) to the
    // voxel owning the parameters just after t, without passing u_hi: the
    // largest e in [u, u_hi] with Tk(e) <= t, by binary search on the exact
    // crossings (they never decrease along the ray).  Needs no position
    // estimate, so a walk keeps no estimate inputs live for it.
    __device__ __forceinline__ int advance_to(int u, float t, int u_hi) const {
        int lo = u, hi = u_hi;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (Tk(mid) <= t) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
};

// Axis a of level `lev`: plane geometry from the per-level table written at
// build time (B, h = fl((A-B)/R), approximate 1/h), ray origin/direction
// component and its correctly rounded reciprocal r = fl(1/d).
__device__ __forceinline__ Axis load_axis(const float *geom, int lev, int a, int R, float o, float d, float r) {
    const float *G = geom + 12 * lev;
    Axis x;
    x.B = G[a];
    x.h = G[3 + a];
    x.inv_h = G[6 + a];
    x.o = o;
    x.d = d;
    x.r = r;
    x.R = R;
    x.pos = d > 0.0f;
    x.zero = (d == 0.0f) || __builtin_isinf(r);
    return x;
}

// Entry/exit parameters (E, X] of the level box: max over moving axes of the
// first plane crossing, min of the last; zero axes must hold o inside.
// Returns false when the level is missed (or the interval is empty).
__device__ __forceinline__ bool level_span(const Axis &ax, const Axis &ay, const Axis &az, float &E, float &X) {
    E = -__builtin_huge_valf();
    X = __builtin_huge_valf();
    const Axis *axes[3] = {&ax, &ay, &az};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const Axis &A = *axes[a];
        if (A.zero) {
            int v = A.zero_voxel();
            if (v < 0 || v >= A.R) return false;
        } else {
            E = fmaxf(E, A.Tk(0));
            X = fminf(X, A.Tk(A.R));
        }
    }
    return E < X;
}

// ---------------------------------------------------------------- lattice

// Sample parameters t_n (Sec. 3): constant step t_n = fl(near + fl(n*dt)),
// or the growing step read from a table t_0..t_{n_tab-1} built by the
// recurrence t_{n+1} = fl(t_n + max(fl(t_n*cone), dt_min)); the table ends
// with the first value past far.
struct Lattice {
    float tmin, tmax, dt;
    const float *tab;   // growing step only
    int32_t n_tab;
    bool cone;

    __device__ __forceinline__ float t(int n) const {
        if (cone) return tab[n];
        return __fadd_rn(tmin, __fmul_rn((float)n, dt));
    }
    // smallest n >= 0 with t_n > a
    __device__ __forceinline__ int first_above(float a) const {
        if (!(a >= tmin)) return 0;
        if (cone) {
            int lo = 0, hi = n_tab - 1;   // tab[n_tab-1] > tmax >= any a asked
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (tab[mid] > a) hi = mid;
                else lo = mid + 1;
            }
            return lo;
        }
        float est = (a - tmin) * __builtin_amdgcn_rcpf(dt);   // estimate only
        est = fminf(fmaxf(est, 0.0f), 16777216.0f);
        int n = (int)est + 1;
        while (n > 0 && t(n - 1) > a) --n;
        while (!(t(n) > a)) ++n;
        return n;
    }
};

}  // namespace ogv
