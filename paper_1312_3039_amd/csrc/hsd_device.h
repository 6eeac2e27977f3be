// Device building blocks shared by the solver kernels: wavefront and
// workgroup reductions, the bounded team barrier, row-group SpMV helpers and
// the cone projections (nonnegative, second-order, PSD by Jacobi in LDS,
// exponential and power cones and their duals).  gfx950: 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hsd_internal.h"

namespace hsd {

constexpr int WAVE = 64;
constexpr int MAX_WAVES = 16;  // 1024 threads per workgroup at most

// ----------------------------------------------------------------------------
// reductions (fixed order: deterministic for a fixed launch shape)
// ----------------------------------------------------------------------------

// Cross-lane moves without LDS traffic: DPP within rows of 16 lanes
// (quad permutations and mirrors) and the gfx950 permlane swaps between
// rows (16 lanes apart) and halves (32 lanes apart).  4- and 8-byte types;
// an 8-byte value moves as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned x) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "dpp_move: 4- or 8-byte values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_u32<CTRL>(__builtin_bit_cast(unsigned, v)));
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = dpp_u32<CTRL>((unsigned)b), hi = dpp_u32<CTRL>((unsigned)(b >> 32));
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}
// For lane pairs 16 (H32 = false) or 32 (H32 = true) lanes apart: lo gets
// the value of the lower lane of the pair and hi that of the upper one, in
// both lanes of the pair.
template <bool H32>
__device__ __forceinline__ void swap_u32(unsigned x, unsigned &lo, unsigned &hi) {
    if constexpr (H32) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        lo = r[0];
        hi = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        lo = r[0];
        hi = r[1];
    }
}
template <bool H32, typename T>
__device__ __forceinline__ void lane_pair(T v, T &lo, T &hi) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "lane_pair: 4- or 8-byte values");
    if constexpr (sizeof(T) == 4) {
        unsigned a, b;
        swap_u32<H32>(__builtin_bit_cast(unsigned, v), a, b);
        lo = __builtin_bit_cast(T, a);
        hi = __builtin_bit_cast(T, b);
    } else {
        const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
        unsigned l0, h0, l1, h1;
        swap_u32<H32>((unsigned)w, l0, h0);
        swap_u32<H32>((unsigned)(w >> 32), l1, h1);
        lo = __builtin_bit_cast(T, ((unsigned long long)l1 << 32) | l0);
        hi = __builtin_bit_cast(T, ((unsigned long long)h1 << 32) | h0);
    }
}

// Sum within aligned groups of L lanes (L a power of two, 1..64): pairs at
// distance 1, 2 (quad permutations), then the two halves of 8 and of 16
// lanes (mirrors), then rows 16 and halves 32 lanes apart (permlane swaps).
// Both lanes of every pair add the same two values, so every lane of a
// group ends with the same bits.  Every lane of the wavefront must call it.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int L) {
    if (L >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    if (L >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    if (L >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
    if (L >= 16) v += dpp_move<0x140>(v); // row_mirror
    if (L >= 32) {
        T a, b;
        lane_pair<false>(v, a, b);
        v = a + b;
    }
    if (L >= 64) {
        T a, b;
        lane_pair<true>(v, a, b);
        v = a + b;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T group_max(T v, int L) {
    for (int off = L >> 1; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, WAVE);
        v = o > v ? o : v;
    }
    return v;
}

// Workgroup sum of NV values held in vals[0..NV), broadcast to every thread.
// red: LDS scratch of NV * MAX_WAVES elements.  Every thread of the
// workgroup must call it.
// A value that every lane of the wave holds equal, moved to scalar
// registers (the compiler cannot prove that values read back from LDS or
// from one global address are uniform, and would keep them in VGPRs).
__device__ __forceinline__ double uniform(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ unsigned uniform(unsigned x) { return __builtin_amdgcn_readfirstlane(x); }

template <int NV, typename T>
__device__ __forceinline__ void block_sum(T *vals, T *red) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        T s = group_sum(vals[k], WAVE);
        if (lane == 0) red[k * MAX_WAVES + wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        T s = T(0);
        for (int w = 0; w < nw; ++w) s += red[k * MAX_WAVES + w];
        vals[k] = uniform(s);  // the same total in every thread
    }
    __syncthreads();
}

// True in every thread when pred is true in any thread of the workgroup.
// scr: LDS scratch of MAX_WAVES words, free again when the call returns.
__device__ __forceinline__ bool block_any(bool pred, unsigned long long *scr) {
    const unsigned long long b = __ballot(pred);
    if ((threadIdx.x & (WAVE - 1)) == 0) scr[threadIdx.x / WAVE] = b;
    __syncthreads();
    unsigned long long a = 0;
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) a |= scr[w];
    __syncthreads();
    return a != 0;
}

// ----------------------------------------------------------------------------
// team barrier: all workgroups of a cooperative launch (or one workgroup)
// ----------------------------------------------------------------------------

// Bounded wait: a workgroup that spins this many times gives up and sets the
// abort flag, which makes every other waiter give up too, so every wave of
// the launch always reaches the end of the kernel.
constexpr unsigned SPIN_LIMIT = 1u << 23;

// Words of the barrier area (unsigned, zeroed before each launch).  The
// per-XCD counters sit on lines of their own.
constexpr int BAR_WORDS = 1024;
constexpr int BAR_COUNT = 0;     // team arrivals (XCD leaders)
constexpr int BAR_ABORT = 2;     // abort flag
constexpr int BAR_REG = 4;       // registrations at team_init
constexpr int BAR_XCD = 32;      // arrivals of XCD x at BAR_XCD + 32 x
constexpr int BAR_MEMBERS = 544; // workgroups on XCD x at BAR_MEMBERS + x
constexpr int MAX_XCD = 16;

// XCD (XCC) that this wave runs on: hardware register XCC_ID, bits [3:0].
__device__ __forceinline__ unsigned xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u;
}

struct Team {
    int rank;                    // workgroup index inside the team
    int size;                    // workgroups in the team
    unsigned *bar;               // BAR_WORDS words (device, zeroed before launch)
    mutable unsigned epoch = 0;  // team barriers this workgroup has entered
    unsigned xcc = 0;            // this workgroup's XCD
    unsigned nx = 0;             // team workgroups on that XCD
    unsigned nxcd = 0;           // XCDs with team workgroups
};

__device__ __forceinline__ bool bar_wait(unsigned *word, unsigned target, unsigned *abrt) {
    unsigned spins = 0;
    while ((int)(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
        if ((spins & 15u) == 15u && __hip_atomic_load(abrt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return false;
        if (++spins > SPIN_LIMIT) {
            __hip_atomic_store(abrt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Once per launch, before the first team_sync: every workgroup registers on
// its XCD, and learns how many team workgroups share that XCD and how many
// XCDs the team spans.  Returns false if the team aborted.
__device__ __forceinline__ bool team_init(Team &tm) {
    if (tm.size == 1) return true;
    __shared__ unsigned s_init[3];
    if (threadIdx.x == 0) {
        unsigned *bar = tm.bar;
        const unsigned x = xcc_id();
        __hip_atomic_fetch_add(bar + BAR_MEMBERS + x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(bar + BAR_REG, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = bar_wait(bar + BAR_REG, (unsigned)tm.size, bar + BAR_ABORT) ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unsigned nxcd = 0;
        for (int k = 0; k < MAX_XCD; ++k)
            nxcd += __hip_atomic_load(bar + BAR_MEMBERS + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        s_init[0] = x;
        s_init[1] = __hip_atomic_load(bar + BAR_MEMBERS + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_init[2] = ok ? nxcd : 0u;
    }
    __syncthreads();
    tm.xcc = s_init[0];
    tm.nx = s_init[1];
    tm.nxcd = s_init[2];
    __syncthreads();
    return tm.nxcd != 0;
}

// Returns false once the team has been aborted.
//
// Two levels: a workgroup arrives on its XCD's counter; the last of the
// XCD's workgroups to arrive writes that XCD's L2 back and arrives on the
// team counter; everybody waits on the team counter.  The counters only
// grow during a launch: barrier number e (from 1) is complete on XCD x when
// its counter reaches e * nx, and for the team when the team counter
// reaches e * nxcd (signed differences, so the counters may wrap).
//
// Memory ordering on gfx950 (eight XCDs, each with its own L2, not coherent
// with the others): every wave first waits for its own global stores to be
// acknowledged, so they sit in its XCD's L2 before its workgroup arrives.
// The L2 write-back is a whole-cache operation, so the one issued by the
// XCD's last arriver (an agent-scope release fence) writes back the stores
// of every workgroup on that XCD; issuing one per XCD instead of one per
// workgroup avoids serialising a dozen write-backs in each L2.  Waiting uses
// relaxed agent-scope loads, which read the coherent copy without
// invalidating any cache; a single agent-scope acquire fence after the wait
// invalidates this workgroup's stale L1 and L2 lines once.  An acquire load
// inside the spin loop would invalidate the XCD's L2 on every poll and
// starve the workgroups still computing.
__device__ __forceinline__ bool team_sync(const Team &tm) {
    if (tm.size == 1) {
        __syncthreads();
        return true;
    }
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    tm.epoch += 1u;
    if (threadIdx.x == 0) {
        unsigned *bar = tm.bar;
        const unsigned before = __hip_atomic_fetch_add(bar + BAR_XCD + 32 * tm.xcc, 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        if (before + 1u == tm.epoch * tm.nx) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(bar + BAR_COUNT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const int ok = bar_wait(bar + BAR_COUNT, tm.epoch * tm.nxcd, bar + BAR_ABORT) ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Partition [0, total) into `parts` contiguous chunks; chunk r.
__device__ __forceinline__ void split_range(int64_t total, int parts, int r, int64_t &a, int64_t &b) {
    a = total * r / parts;
    b = total * (r + 1) / parts;
}

// ----------------------------------------------------------------------------
// exponential cone (Sect. 6.1 definitions)
// ----------------------------------------------------------------------------

__device__ __forceinline__ double exp_capped(double a) { return a > 700.0 ? HUGE_VAL : exp(a); }

__device__ __forceinline__ bool dev_in_exp(double x, double y, double z) {
    if (y > 0.0 && y * exp_capped(x / y) <= z) return true;
    return x <= 0.0 && y == 0.0 && z >= 0.0;
}

__device__ __forceinline__ bool dev_in_exp_dual(double u, double v, double w) {
    if (u < 0.0 && -u * exp_capped(v / u) <= 2.718281828459045235 * w) return true;
    return u == 0.0 && v >= 0.0 && w >= 0.0;
}

// Sign of the optimality condition for the nearest point to (x0,y0,z0) on
// the ray y*(r, 1, e^r): with d = (r,1,e^r), d' = (1,0,e^r) the condition is
// <v,d'>|d|^2 = <v,d><d,d'>, which expands to
//   (x0 - r y0) + e^{2r}((1-r) x0 - y0) + z0 e^r (r^2 - r + 1) = 0.
// For r > 0 the expression is multiplied by e^{-2r} (same sign).
__device__ __forceinline__ double exp_root_fn(double r, double x0, double y0, double z0) {
    const double q = r * r - r + 1.0;
    if (r > 0.0) {
        const double e = exp(-r);
        return (x0 - r * y0) * e * e + ((1.0 - r) * x0 - y0) + z0 * e * q;
    }
    const double e = exp(r);
    return (x0 - r * y0) + e * e * ((1.0 - r) * x0 - y0) + z0 * e * q;
}

// Nearest point to v on the ray through (r, 1, e^r); direction rescaled by
// e^{-r} when r > 0.
__device__ __forceinline__ void exp_ray_point(double r, double x0, double y0, double z0,
                                              double &px, double &py, double &pz) {
    double d0, d1, d2;
    if (r > 0.0) {
        const double e = exp(-r);
        d0 = r * e; d1 = e; d2 = 1.0;
    } else {
        d0 = r; d1 = 1.0; d2 = exp(r);
    }
    double ip = x0 * d0 + y0 * d1 + z0 * d2;
    double t = (ip > 0.0 ? ip : 0.0) / (d0 * d0 + d1 * d1 + d2 * d2);
    px = t * d0; py = t * d1; pz = t * d2;
}

// Projection onto K_exp.  Cases: inside -> itself; inside the polar -> 0;
// x0 <= 0 and y0 <= 0 -> (x0, 0, max(z0, 0)); otherwise the nearest point
// of the curved boundary, whose ratio r = x/y lies where r x0 > x0 - y0 and
// r y0 < x0 (conditions for v = y d(r) + c n(r) with y, c > 0, n the surface
// normal); open ends of that interval are closed by doubling, the root is
// bisected to full precision, and the nearest of the candidate points
// (root, bracket ends, face point, apex) is returned.
__device__ void proj_exp_dev(double &x, double &y, double &z) {
    const double x0 = x, y0 = y, z0 = z;
    if (dev_in_exp(x0, y0, z0)) return;
    if (dev_in_exp_dual(-x0, -y0, -z0)) { x = 0.0; y = 0.0; z = 0.0; return; }
    if (x0 <= 0.0 && y0 <= 0.0) { y = 0.0; z = z0 > 0.0 ? z0 : 0.0; return; }
    double lo = -HUGE_VAL, hi = HUGE_VAL;
    if (x0 > 0.0) lo = fmax(lo, 1.0 - y0 / x0);
    else if (x0 < 0.0) hi = fmin(hi, 1.0 - y0 / x0);
    if (y0 > 0.0) hi = fmin(hi, x0 / y0);
    else if (y0 < 0.0) lo = fmax(lo, x0 / y0);
    if (isinf(lo) && isinf(hi)) { lo = -1.0; hi = 1.0; }
    if (isinf(hi)) {
        double step = 1.0;
        hi = lo + step;
        while (exp_root_fn(hi, x0, y0, z0) > 0.0 && step < 1e6) { step *= 2.0; hi = lo + step; }
    }
    if (isinf(lo)) {
        double step = 1.0;
        lo = hi - step;
        while (exp_root_fn(lo, x0, y0, z0) < 0.0 && step < 1e6) { step *= 2.0; lo = hi - step; }
    }
    // candidates: apex, face point, bracket ends, root
    double bx = 0.0, by = 0.0, bz = 0.0;
    double best = x0 * x0 + y0 * y0 + z0 * z0;
    auto consider = [&](double px, double py, double pz) {
        double dx = px - x0, dy = py - y0, dz = pz - z0;
        double dd = dx * dx + dy * dy + dz * dz;
        if (dd < best) { best = dd; bx = px; by = py; bz = pz; }
    };
    consider(x0 < 0.0 ? x0 : 0.0, 0.0, z0 > 0.0 ? z0 : 0.0);
    double px, py, pz;
    exp_ray_point(lo, x0, y0, z0, px, py, pz); consider(px, py, pz);
    exp_ray_point(hi, x0, y0, z0, px, py, pz); consider(px, py, pz);
    double flo = exp_root_fn(lo, x0, y0, z0);
    double fhi = exp_root_fn(hi, x0, y0, z0);
    if (flo != 0.0 && fhi != 0.0 && ((flo > 0.0) != (fhi > 0.0))) {
        double a = lo, b = hi, fa = flo;
        for (int it = 0; it < 400; ++it) {
            double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            double fm = exp_root_fn(mid, x0, y0, z0);
            if (fm == 0.0) { a = mid; b = mid; break; }
            if ((fm > 0.0) == (fa > 0.0)) { a = mid; fa = fm; } else { b = mid; }
        }
        exp_ray_point(0.5 * (a + b), x0, y0, z0, px, py, pz);
        consider(px, py, pz);
    }
    x = bx; y = by; z = bz;
}

// Projection onto K_exp^* by Moreau: Pi_{K*}(v) = v + Pi_K(-v).
__device__ __forceinline__ void proj_exp_dual_dev(double &x, double &y, double &z) {
    double a = -x, b = -y, c = -z;
    proj_exp_dev(a, b, c);
    x += a; y += b; z += c;
}

// ----------------------------------------------------------------------------
// power cone K_pow^a = {(x, y, z): x^a y^(1-a) >= |z|, x >= 0, y >= 0} and its
// dual {(u, v, w): (u/a)^a (v/(1-a))^(1-a) >= |w|, u >= 0, v >= 0}, a in [0, 1]
// (Sect. 6.1 definitions).  A factor whose exponent is zero is 1.
// ----------------------------------------------------------------------------

__device__ __forceinline__ double pow_factor(double t, double e) { return e == 0.0 ? 1.0 : pow(t, e); }

__device__ __forceinline__ bool dev_in_pow(double x, double y, double z, double a) {
    return x >= 0.0 && y >= 0.0 && pow_factor(x, a) * pow_factor(y, 1.0 - a) >= fabs(z);
}

__device__ __forceinline__ bool dev_in_pow_dual(double u, double v, double w, double a) {
    if (u < 0.0 || v < 0.0) return false;
    const double fu = a == 0.0 ? 1.0 : pow(u / a, a);
    const double fv = a == 1.0 ? 1.0 : pow(v / (1.0 - a), 1.0 - a);
    return fu * fv >= fabs(w);
}

// Nonnegative root of t^2 - t0 t - c = 0 (c >= 0); for t0 < 0 in the form
// 2c / (s - t0), which avoids the cancellation of (t0 + s) / 2.
__device__ __forceinline__ double pow_root(double t0, double c) {
    const double s = sqrt(t0 * t0 + 4.0 * c);
    return t0 >= 0.0 ? 0.5 * (t0 + s) : 2.0 * c / (s - t0);
}

// Projection onto K_pow^a.  Outside the cone and its polar, with z0 != 0,
// the nearest point lies on the boundary with z = sign(z0) r, 0 < r < |z0|.
// For a fixed r, the stationarity conditions of the distance with the
// multiplier mu = |z0| - r of the constraint x^a y^(1-a) >= r read
// x^2 - x0 x = a r mu and y^2 - y0 y = (1-a) r mu, whose nonnegative roots
// give x(r), y(r); r is where x(r)^a y(r)^(1-a) = r, a sign change of that
// difference over (0, |z0|), found by bisection to full precision.
__device__ void proj_pow_dev(double &x, double &y, double &z, double a) {
    const double x0 = x, y0 = y, z0 = z;
    if (dev_in_pow(x0, y0, z0, a)) return;
    if (dev_in_pow_dual(-x0, -y0, -z0, a)) { x = 0.0; y = 0.0; z = 0.0; return; }
    if (z0 == 0.0) { x = x0 > 0.0 ? x0 : 0.0; y = y0 > 0.0 ? y0 : 0.0; return; }
    const double az = fabs(z0);
    double lo = 0.0, hi = az;
    for (int it = 0; it < 256; ++it) {
        const double r = 0.5 * (lo + hi);
        if (r <= lo || r >= hi) break;
        const double mu = az - r;
        const double xr = pow_root(x0, a * r * mu), yr = pow_root(y0, (1.0 - a) * r * mu);
        if (pow_factor(xr, a) * pow_factor(yr, 1.0 - a) > r) lo = r; else hi = r;
    }
    const double r = 0.5 * (lo + hi);
    const double mu = az - r;
    x = pow_root(x0, a * r * mu);
    y = pow_root(y0, (1.0 - a) * r * mu);
    z = z0 > 0.0 ? r : -r;
}

// Projection onto (K_pow^a)^* by Moreau: Pi_{K*}(v) = v + Pi_K(-v).
__device__ __forceinline__ void proj_pow_dual_dev(double &x, double &y, double &z, double a) {
    double p = -x, q = -y, r = -z;
    proj_pow_dev(p, q, r, a);
    x += p; y += q; z += r;
}

// ----------------------------------------------------------------------------
// PSD cone: cyclic Jacobi in LDS by one workgroup (Golub & Van Loan, the
// parallel-ordering symmetric Jacobi method), then clamp and rebuild.
// ----------------------------------------------------------------------------

// LDS doubles needed for a PSD cone of side d (matrix, eigenvectors,
// rotations, scratch; with warm starts a third d x d product buffer).
__host__ __device__ inline int psd_lds_doubles(int d, bool warm = false) {
    const int dp = d + (d & 1);
    return (warm ? 3 : 2) * dp * (dp + 1) + 3 * (dp / 2) + 2 * MAX_WAVES + 8;
}

// Largest PSD side whose projections are warm-started (the three d x d
// buffers in LDS beside the rest of the solve kernel's LDS).
constexpr int PSD_WARM_MAX = 64;

// D = op(X) Y for dp x dp matrices in LDS (row stride ld), by the FP64
// matrix cores: 16 x 16 output tiles, one per wavefront at a time, the
// inner dimension in steps of 4 (v_mfma_f64_16x16x4: lane l supplies
// X(i0 + l % 16, k + l / 16) and Y(k + l / 16, j0 + l % 16) and receives
// D(i0 + l / 16 + 4 r, j0 + l % 16), r = 0..3).  Entries beyond dp count as
// zero.  XT: op(X) = X^T; YT: op(Y) = Y^T (D = op(X) op(Y)).
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <bool XT, bool YT = false>
__device__ __forceinline__ void psd_mfma_product(double *D, const double *X, const double *Y, int dp, int ld) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int nt = (dp + 15) / 16;
    for (int t = wid; t < nt * nt; t += nw) {
        const int i0 = (t / nt) * 16, j0 = (t % nt) * 16;
        const int ia = i0 + (lane & 15), jb = j0 + (lane & 15), kl = lane >> 4;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < dp; k += 4) {
            const int kk = k + kl;
            double a = 0.0, b = 0.0;
            if (ia < dp && kk < dp) a = XT ? X[kk * ld + ia] : X[ia * ld + kk];
            if (jb < dp && kk < dp) b = YT ? Y[jb * ld + kk] : Y[kk * ld + jb];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + kl + 4 * r;
            if (i < dp && jb < dp) D[i * ld + jb] = acc[r];
        }
    }
}

// A <- V^T A V for the warm start of the Jacobi sweeps (T = A V, then
// V^T T, both on the matrix cores), then exact symmetry for the rotations
// (the mean of the two triangles).  All dp x dp in LDS; every thread of the
// workgroup calls it.  Out of line: it is off the path of programs without
// PSD cones.
__device__ __noinline__ void psd_rotate_into(double *Am, const double *Vm, double *Tm, int dp, int ld) {
    const int tid = threadIdx.x, nt = blockDim.x;
    psd_mfma_product<false>(Tm, Am, Vm, dp, ld);
    __syncthreads();
    psd_mfma_product<true>(Am, Vm, Tm, dp, ld);
    __syncthreads();
    for (int e = tid; e < dp * dp; e += nt) {
        const int i = e / dp, j = e % dp;
        if (i < j) Tm[i * ld + j] = 0.5 * (Am[i * ld + j] + Am[j * ld + i]);
    }
    __syncthreads();
    for (int e = tid; e < dp * dp; e += nt) {
        const int i = e / dp, j = e % dp;
        if (i < j) Am[i * ld + j] = Tm[i * ld + j];
        else if (i > j) Am[i * ld + j] = Tm[j * ld + i];
    }
    __syncthreads();
}

// Projects the scaled-svec vector of side d.  fin(i) gives element i of the
// argument (i < d(d+1)/2); fout(i, p, a) receives the projected value p and
// the argument a of element i.  All threads of the workgroup must call it.
//
// Warm start (vstore given): the eigenvectors found by the previous
// projection of the same cone are kept in vstore (dp x dp).  The argument
// changes little from one update to the next, so with warm set the matrix
// is first rotated into that basis, A <- V^T A V, which leaves it nearly
// diagonal, and the Jacobi sweeps start from V: they converge in a sweep or
// two instead of about ten.  The eigenvectors found are stored back.  The
// projection is the same (unique) point up to rounding.
template <bool WARM = false, typename Fin, typename Fout>
__device__ void proj_psd_block(int d, double *lds, Fin fin, Fout fout, double *vstore = nullptr,
                               bool warm = false) {
    if constexpr (!WARM) vstore = nullptr;
    const int dp = d + (d & 1);
    const int half = dp / 2;
    // rows of Am, Vm (and Tm) are ld = dp + 1 doubles apart: an odd stride,
    // so that the column accesses of a rotation fall in different LDS banks
    const int ld = dp + 1;
    double *Am = lds;
    double *Vm = Am + dp * ld;
    double *cs = Vm + dp * ld;
    double *sn = cs + half;
    int *pq = reinterpret_cast<int *>(sn + half);  // the pairs of a round: p, q
    double *red = sn + 2 * half;
    double *Tm = red + 2 * MAX_WAVES + 8;  // warm start only: dp x ld
    const int tid = threadIdx.x, nt = blockDim.x;
    const double rs2 = 0.70710678118654752440;
    // unpack: svec index of (i, j), i >= j, column-major lower triangle
    for (int e = tid; e < dp * dp; e += nt) {
        int i = e / dp, j = e % dp;
        double val = 0.0;
        if (i < d && j < d) {
            int r = i > j ? i : j, c = i > j ? j : i;
            int idx = c * d - (c * (c - 1)) / 2 + (r - c);
            val = fin(idx);
            if (r != c) val *= rs2;
        }
        Am[i * ld + j] = val;
        Vm[i * ld + j] = (WARM && vstore != nullptr && warm) ? vstore[e] : ((i == j) ? 1.0 : 0.0);
    }
    __syncthreads();
    if constexpr (WARM) {
        if (vstore != nullptr && warm) psd_rotate_into(Am, Vm, Tm, dp, ld);
    }
    double fro[1] = {0.0};
    for (int e = tid; e < dp * dp; e += nt) {
        const double a = Am[(e / dp) * ld + e % dp];
        fro[0] += a * a;
    }
    block_sum<1>(fro, red);
    // sweeps until the off-diagonal part is below 1e-12 of the matrix
    // (Frobenius norms): the projection is then exact to about that
    // relative accuracy, far below any tolerance of the method
    const double stop2 = fro[0] * 1e-24;
    // this thread's first element (pr, k) of a round's half * dp, and the
    // step nt = pr_step * dp + k_step
    const int pr0 = tid / dp, k0 = tid % dp, pr_step = nt / dp, k_step = nt % dp;
    // the same for the half x half blocks (bi, bj) of a round
    const int bi0 = tid / half, bj0 = tid % half, bi_step = nt / half, bj_step = nt % half;
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off[1] = {0.0};
        for (int e = tid; e < dp * dp; e += nt) {
            int i = e / dp, j = e % dp;
            if (i != j) off[0] += Am[i * ld + j] * Am[i * ld + j];
        }
        block_sum<1>(off, red);
        if (!(off[0] > stop2)) break;
        for (int round = 0; round < dp - 1; ++round) {
            // round-robin pairing: position 0 fixed, the rest rotate; the
            // pair (p, q) of slot tid goes to LDS with its rotation
            if (tid < half) {
                int a = (tid == 0) ? 0 : ((tid - 1 + round) % (dp - 1)) + 1;
                int bpos = dp - 1 - tid;
                int b = ((bpos - 1 + round) % (dp - 1)) + 1;
                int p = a < b ? a : b, q = a < b ? b : a;
                pq[2 * tid] = p;
                pq[2 * tid + 1] = q;
                double c = 1.0, s = 0.0;
                double apq = Am[p * ld + q];
                if (apq != 0.0) {
                    double theta = (Am[q * ld + q] - Am[p * ld + p]) / (2.0 * apq);
                    double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            // A <- J^T A J by 2 x 2 blocks (the rows of pair bi, the columns
            // of pair bj: the row rotation, then the column rotation, as
            // the rows-then-columns order computes them), and V <- V J by
            // the element pairs (k, pr); one barrier for both.  The blocks
            // and element pairs are walked without integer division.
            for (int e = tid, bi = bi0, bj = bj0; e < half * half; e += nt, bi += bi_step, bj += bj_step) {
                if (bj >= half) { bj -= half; ++bi; }
                const int pi = pq[2 * bi], qi = pq[2 * bi + 1], pj = pq[2 * bj], qj = pq[2 * bj + 1];
                const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
                const double a = Am[pi * ld + pj], b = Am[pi * ld + qj];
                const double g = Am[qi * ld + pj], h = Am[qi * ld + qj];
                const double a1 = ci * a - si * g, g1 = si * a + ci * g;
                const double b1 = ci * b - si * h, h1 = si * b + ci * h;
                Am[pi * ld + pj] = cj * a1 - sj * b1;
                Am[pi * ld + qj] = sj * a1 + cj * b1;
                Am[qi * ld + pj] = cj * g1 - sj * h1;
                Am[qi * ld + qj] = sj * g1 + cj * h1;
            }
            for (int e = tid, pr = pr0, k = k0; e < half * dp; e += nt, pr += pr_step, k += k_step) {
                if (k >= dp) { k -= dp; ++pr; }
                const int p = pq[2 * pr], q = pq[2 * pr + 1];
                double c = cs[pr], s = sn[pr];
                double vp = Vm[k * ld + p], vq = Vm[k * ld + q];
                Vm[k * ld + p] = c * vp - s * vq;
                Vm[k * ld + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    // eigenvalues are on the diagonal of Am, eigenvectors in the columns of Vm
    // (stored for the next warm start).  Rebuild P = V diag(max(lambda, 0)) V^T
    // as W W^T on the matrix cores, W = V diag(sqrt(max(lambda, 0))) in place
    // of V, into Am; then write its lower triangle in scaled svec.
    for (int e = tid; e < dp * dp; e += nt) {
        const int i = e / dp, k = e % dp;
        const double v = Vm[i * ld + k];
        if constexpr (WARM) {
            if (vstore != nullptr) vstore[e] = v;
        }
        const double lam = Am[k * ld + k];
        Vm[i * ld + k] = lam > 0.0 ? v * sqrt(lam) : 0.0;
    }
    __syncthreads();
    psd_mfma_product<false, true>(Am, Vm, Vm, dp, ld);
    __syncthreads();
    const int L = d * (d + 1) / 2;
    for (int idx = tid; idx < L; idx += nt) {
        // invert the svec index: column c, row r >= c
        int c = 0, rem = idx;
        while (rem >= d - c) { rem -= d - c; ++c; }
        int r = c + rem;
        const double acc = Am[r * ld + c];
        double a = fin(idx);
        fout(idx, (r == c) ? acc : acc * 1.41421356237309504880, a);
    }
    __syncthreads();
}

}  // namespace hsd
