// lsm_kernels.hip -- HIP kernels (gfx950) of the lattice spring model step.
//
// One workgroup owns a 64 x 4 tile of lattice sites (one wavefront per row
// segment, so every state load of a wavefront is 64 consecutive sites).
// Each thread owns one site (particle) and gathers the forces of all its
// incident springs in a fixed direction order, so the force sum is
// deterministic and independent of the launch shape, and no atomics are
// needed: a spring shared by particles p and q is evaluated by both, from
// bitwise-negated inputs, so both reach the same break decision and exactly
// opposite forces (Eq. 2).  Each particle keeps its own copy of the broken
// bit of each incident spring; the owner (lower id, forward direction) logs
// the break event.
//
// The step kernel fuses, per site: spring force with the critical-stretch
// test (Eq. 1-2; Section 2.3 force routine), force accumulation, and the
// velocity Verlet update in the half-step form (Eq. 3-5, Section 2.2) with
// viscous damping.  Displacements u = x - X0 are stored (X0 is implied by
// the site index), double-buffered between steps; velocities are updated in
// place.  In the FP32 mode forces are FP32 and displacements are kept as a
// compensated (hi, lo) FP32 pair; springs whose squared length is within a
// narrow band of rc^2 are re-tested in FP64 from the compensated state.
#include <math.h>

#include <type_traits>

#include "lsm_internal.h"

namespace lsm {
namespace {

// Relative band on r^2 below rc^2 inside which the FP32 break decision is
// handed to FP64.  FP32 errors of r^2 here are below 1e-6 relative.
constexpr float kBand2 = 3.0e-5f;
constexpr double kHalfSqrt3 = 0.86602540378443864676;

// ------------------------------------------------------------ state layout
template <int DIM, int PREC>
struct State;

// 2D, FP32 compensated: u = (x_hi, y_hi, x_lo, y_lo) as float4, v float2.
template <>
struct State<2, 1> {
    using R = float;
    __device__ static void load_u(const void *U, int g, int64_t, float hi[2], float lo[2]) {
        const float4 t = reinterpret_cast<const float4 *>(U)[g];
        hi[0] = t.x; hi[1] = t.y; lo[0] = t.z; lo[1] = t.w;
    }
    __device__ static void store_u(void *U, int g, int64_t, const float hi[2], const float lo[2]) {
        reinterpret_cast<float4 *>(U)[g] = make_float4(hi[0], hi[1], lo[0], lo[1]);
    }
    __device__ static void load_v(const void *V, int g, int64_t, float v[2]) {
        const float2 t = reinterpret_cast<const float2 *>(V)[g];
        v[0] = t.x; v[1] = t.y;
    }
    __device__ static void store_v(void *V, int g, int64_t, const float v[2]) {
        reinterpret_cast<float2 *>(V)[g] = make_float2(v[0], v[1]);
    }
};

// 2D, FP64: u and v as double2; the low part is identically zero.
template <>
struct State<2, 0> {
    using R = double;
    __device__ static void load_u(const void *U, int g, int64_t, double hi[2], double lo[2]) {
        const double2 t = reinterpret_cast<const double2 *>(U)[g];
        hi[0] = t.x; hi[1] = t.y; lo[0] = 0.0; lo[1] = 0.0;
    }
    __device__ static void store_u(void *U, int g, int64_t, const double hi[2], const double *) {
        reinterpret_cast<double2 *>(U)[g] = make_double2(hi[0], hi[1]);
    }
    __device__ static void load_v(const void *V, int g, int64_t, double v[2]) {
        const double2 t = reinterpret_cast<const double2 *>(V)[g];
        v[0] = t.x; v[1] = t.y;
    }
    __device__ static void store_v(void *V, int g, int64_t, const double v[2]) {
        reinterpret_cast<double2 *>(V)[g] = make_double2(v[0], v[1]);
    }
};

// 3D, FP32 compensated: u as a float4 plane (x_hi, y_hi, z_hi, x_lo) followed
// by a float2 plane (y_lo, z_lo) -- two loads per neighbour; v three planes.
template <>
struct State<3, 1> {
    using R = float;
    __device__ static void load_u(const void *U, int g, int64_t ns, float hi[3], float lo[3]) {
        const float4 a = reinterpret_cast<const float4 *>(U)[g];
        const float2 b = reinterpret_cast<const float2 *>(reinterpret_cast<const float4 *>(U) + ns)[g];
        hi[0] = a.x; hi[1] = a.y; hi[2] = a.z; lo[0] = a.w; lo[1] = b.x; lo[2] = b.y;
    }
    __device__ static void store_u(void *U, int g, int64_t ns, const float hi[3], const float lo[3]) {
        reinterpret_cast<float4 *>(U)[g] = make_float4(hi[0], hi[1], hi[2], lo[0]);
        reinterpret_cast<float2 *>(reinterpret_cast<float4 *>(U) + ns)[g] = make_float2(lo[1], lo[2]);
    }
    __device__ static void load_v(const void *V, int g, int64_t ns, float v[3]) {
        const float *P = reinterpret_cast<const float *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = P[c * ns + g];
    }
    __device__ static void store_v(void *V, int g, int64_t ns, const float v[3]) {
        float *P = reinterpret_cast<float *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) P[c * ns + g] = v[c];
    }
    // the same with 32-bit byte offsets from the array base (compact
    // arrays of fewer than 2^32 bytes)
    __device__ static void load_u(const void *U, uint32_t g, uint32_t ns, float hi[3], float lo[3]) {
        const char *b = static_cast<const char *>(U);
        const float4 a = *reinterpret_cast<const float4 *>(b + g * 16u);
        const float2 c = *reinterpret_cast<const float2 *>(b + (ns * 16u + g * 8u));
        hi[0] = a.x; hi[1] = a.y; hi[2] = a.z; lo[0] = a.w; lo[1] = c.x; lo[2] = c.y;
    }
    __device__ static void store_u(void *U, uint32_t g, uint32_t ns, const float hi[3], const float lo[3]) {
        char *b = static_cast<char *>(U);
        *reinterpret_cast<float4 *>(b + g * 16u) = make_float4(hi[0], hi[1], hi[2], lo[0]);
        *reinterpret_cast<float2 *>(b + (ns * 16u + g * 8u)) = make_float2(lo[1], lo[2]);
    }
    __device__ static void load_v(const void *V, uint32_t g, uint32_t ns, float v[3]) {
        const char *b = static_cast<const char *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = *reinterpret_cast<const float *>(b + (uint32_t(c) * ns + g) * 4u);
    }
    __device__ static void store_v(void *V, uint32_t g, uint32_t ns, const float v[3]) {
        char *b = static_cast<char *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) *reinterpret_cast<float *>(b + (uint32_t(c) * ns + g) * 4u) = v[c];
    }
};

// 3D, FP64: three planes for u and for v.
template <>
struct State<3, 0> {
    using R = double;
    __device__ static void load_u(const void *U, int g, int64_t ns, double hi[3], double lo[3]) {
        const double *P = reinterpret_cast<const double *>(U);
#pragma unroll
        for (int c = 0; c < 3; ++c) { hi[c] = P[c * ns + g]; lo[c] = 0.0; }
    }
    __device__ static void store_u(void *U, int g, int64_t ns, const double hi[3], const double *) {
        double *P = reinterpret_cast<double *>(U);
#pragma unroll
        for (int c = 0; c < 3; ++c) P[c * ns + g] = hi[c];
    }
    __device__ static void load_v(const void *V, int g, int64_t ns, double v[3]) {
        const double *P = reinterpret_cast<const double *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = P[c * ns + g];
    }
    __device__ static void store_v(void *V, int g, int64_t ns, const double v[3]) {
        double *P = reinterpret_cast<double *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) P[c * ns + g] = v[c];
    }
    __device__ static void load_u(const void *U, uint32_t g, uint32_t ns, double hi[3], double lo[3]) {
        const char *b = static_cast<const char *>(U);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hi[c] = *reinterpret_cast<const double *>(b + (uint32_t(c) * ns + g) * 8u);
            lo[c] = 0.0;
        }
    }
    __device__ static void store_u(void *U, uint32_t g, uint32_t ns, const double hi[3], const double *) {
        char *b = static_cast<char *>(U);
#pragma unroll
        for (int c = 0; c < 3; ++c) *reinterpret_cast<double *>(b + (uint32_t(c) * ns + g) * 8u) = hi[c];
    }
    __device__ static void load_v(const void *V, uint32_t g, uint32_t ns, double v[3]) {
        const char *b = static_cast<const char *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = *reinterpret_cast<const double *>(b + (uint32_t(c) * ns + g) * 8u);
    }
    __device__ static void store_v(void *V, uint32_t g, uint32_t ns, const double v[3]) {
        char *b = static_cast<char *>(V);
#pragma unroll
        for (int c = 0; c < 3; ++c) *reinterpret_cast<double *>(b + (uint32_t(c) * ns + g) * 8u) = v[c];
    }
};

// ------------------------------------------------------- lattice geometry
// Directions: forward ones first, in canonical spring order, then their
// opposites in the same order (opposite of d is d + NF).
template <int DIM>
struct Geo;

// Triangular packing, odd rows shifted by +a/2.  Directions: E, UL, UR, W,
// DR, DL.  Column offset = base + parity * adj, row offset = drow.
template <>
struct Geo<2> {
    static constexpr int ND = 6, NF = 3;
    using Mask = uint8_t;
    __device__ static int di(int d, int par) {
        constexpr int base[6] = {1, -1, 0, -1, 0, -1};
        constexpr int adj[6] = {0, 1, 1, 0, 1, 1};
        return base[d] + par * adj[d];
    }
    __device__ static int dj(int d) {
        constexpr int v[6] = {0, 1, 1, 0, -1, -1};
        return v[d];
    }
    __device__ static int dk(int) { return 0; }
    // lattice vector in units of (a, (sqrt3/2) a)
    __device__ static double ex(int d) {
        constexpr double v[6] = {1.0, -0.5, 0.5, -1.0, 0.5, -0.5};
        return v[d];
    }
    __device__ static double ey(int d) {
        constexpr double v[6] = {0.0, 1.0, 1.0, 0.0, -1.0, -1.0};
        return v[d];
    }
    __device__ static int geom(int) { return 0; }
};

// Simple cubic, 3 face + 6 edge forward directions.
template <>
struct Geo<3> {
    static constexpr int ND = 18, NF = 9;
    using Mask = uint32_t;
    __device__ static int off(int d, int c) {
        constexpr int f[9][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {1, 1, 0}, {-1, 1, 0},
                                 {1, 0, 1},  {-1, 0, 1}, {0, 1, 1},  {0, -1, 1}};
        return d < 9 ? f[d][c] : -f[d - 9][c];
    }
    __device__ static int di(int d, int) { return off(d, 0); }
    __device__ static int dj(int d) { return off(d, 1); }
    __device__ static int dk(int d) { return off(d, 2); }
    __device__ static int geom(int d) { return (d % 9) < 3 ? 0 : 1; }
};

template <int PREC>
struct TT;
template <>
struct TT<1> {
    // k, k r0, r^2 above which the break test is redone in FP64 (just
    // below rc^2), r0
    using type = float4;
    __device__ static type make(const TypeRec &t) {
        return make_float4(t.k32, t.kr0_32, t.rc2_32 - kBand2 * t.rc2_32, t.r0_32);
    }
};
struct D4 {
    double x, y, z, w;
};
template <>
struct TT<0> {
    using type = D4;  // k, r0, rc, rc^2
    __device__ static type make(const TypeRec &t) { return D4{t.k64, t.r0_64, t.rc64, t.rc64 * t.rc64}; }
};

__device__ inline void comp_add(float &hi, float &lo, float delta) {
    // compensated accumulation: hi + lo absorbs delta, the rounding error of
    // the high sum is carried exactly in lo (two-sum)
    const float y = delta + lo;
    const float t = hi + y;
    const float bp = t - hi;
    lo = (hi - (t - bp)) + (y - bp);
    hi = t;
}
__device__ inline void comp_add(double &hi, double &, double delta) { hi = hi + delta; }
// the same with delta = a b, the product rounded once with the low part
__device__ inline void comp_add_fma(float &hi, float &lo, float a, float b) {
    const float y = fmaf(a, b, lo);
    const float t = hi + y;
    const float bp = t - hi;
    lo = (hi - (t - bp)) + (y - bp);
    hi = t;
}

// 1/sqrt(x) for a positive normal x: the hardware estimate y0 refined by
// the second-order expansion of (1 - e)^(-1/2), e = 1 - x y0^2:
// y = y0 (1 + e/2 + 3 e^2 / 8), whose error is of order e^3.
__device__ inline double rsqrt_pos(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y0, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Fixed-order workgroup sum of kNumPartials values; result valid in thread 0.
__device__ inline void block_sum(double *vals, double (*lds)[kBlock / 64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < kNumPartials; ++v) {
        const double s = wave_sum(vals[v]);
        if (lane == 0) lds[v][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int v = 0; v < kNumPartials; ++v) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += lds[v][w];
            vals[v] = s;
        }
    }
}

__device__ inline void tile_coords(const StepParams &P, int &i, int &j, int &k, bool &ok) {
    // XCD-aware remap: consecutive blocks go round-robin over the 8 XCDs, so
    // give each XCD one contiguous run of tiles (neighbouring rows share L2).
    const int b = blockIdx.x;
    const int per = P.nblocks >> 3;
    const int tile = (b & 7) * per + (b >> 3);
    ok = tile < P.ntiles;
    const int tx = tile % P.tiles_x;
    const int rest = tile / P.tiles_x;
    const int ty = rest % P.tiles_y;
    const int tz = rest / P.tiles_y;
    i = tx * kTileX + (threadIdx.x & (kTileX - 1));
    j = ty * kTileY + (threadIdx.x / kTileX);
    k = tz;
    ok = ok && i < P.nx && j < P.ny;
}

// Slot of this lane's event in the break log: one atomic per wavefront for
// the lanes logging at this point (their ballot), slots in lane order
// within it.  The log's order across wavefronts depends on scheduling; the
// host sorts it on read.
__device__ inline uint32_t event_slot(Ctl *ctl) {
    const uint64_t act = __ballot(1);
    const int lane = int(__lane_id());
    const int leader = __ffsll(static_cast<unsigned long long>(act)) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&ctl->n_events, uint32_t(__popcll(act)));
    base = uint32_t(__shfl(int(base), leader, 64));
    return base + uint32_t(__popcll(act & ((uint64_t(1) << lane) - 1u)));
}

// Acceleration (F - gamma v) / m of a free particle (v: the half-step velocity).
template <int DIM, int PREC>
__device__ inline void site_acc(const typename State<DIM, PREC>::R *F, const typename State<DIM, PREC>::R *w,
                                double mass, typename State<DIM, PREC>::R inv_mass,
                                typename State<DIM, PREC>::R gam, typename State<DIM, PREC>::R *acc) {
    using R = typename State<DIM, PREC>::R;
    if constexpr (PREC == 1) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] = (F[c] - gam * w[c]) * inv_mass;
    } else {
        const R m = R(mass);
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] = (F[c] - gam * w[c]) / m;
    }
}

// Interior step: close the half kick, open the next one, drift.  In FP32
// the two half kicks are one kick by dt (h + h = dt exactly) and the drift
// product is fused into the compensated sum.
template <int DIM, int PREC>
__device__ inline void mid_kick_drift(typename State<DIM, PREC>::R *uph, typename State<DIM, PREC>::R *upl,
                                      typename State<DIM, PREC>::R *w, const typename State<DIM, PREC>::R *acc,
                                      typename State<DIM, PREC>::R h, typename State<DIM, PREC>::R dt) {
    using R = typename State<DIM, PREC>::R;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        if constexpr (PREC == 1) {
            w[c] = fmaf(dt, acc[c], w[c]);
            comp_add_fma(uph[c], upl[c], dt, w[c]);
        } else {
            const R vfull = w[c] + h * acc[c];
            w[c] = vfull + h * acc[c];
            comp_add(uph[c], upl[c], dt * w[c]);
        }
    }
}

// Velocity Verlet in the half-step form (Eq. 3-5) with viscous damping
// evaluated with the half-step velocity, for one free particle; grips stay
// clamped.  On entry w is the particle's stored velocity (full step at the
// start of an increment, half step otherwise); F is the spring force at the
// current positions.
// Where a site's new state goes: by site index (gather kernel) ...
template <int DIM, int PREC>
struct SiteStore {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    int g;
    int64_t ns;
    __device__ void u(void *U, const R *hi, const R *lo) const { S::store_u(U, g, ns, hi, lo); }
    __device__ void v(void *V, const R *w) const { S::store_v(V, g, ns, w); }
};

// ... or by 32-bit byte offsets in the compact 3D arrays ...
template <int DIM, int PREC>
struct SiteStore32 {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    uint32_t g, ns;
    __device__ void u(void *U, const R *hi, const R *lo) const { S::store_u(U, g, ns, hi, lo); }
    __device__ void v(void *V, const R *w) const { S::store_v(V, g, ns, w); }
};

// ... or in the compact 3D arrays, addressed by 32-bit byte offsets (arrays
// of fewer than 2^32 bytes).  Displacements are two planes of ns records:
// 16-byte (FP64 x, y; FP32-compensated x_hi, y_hi, z_hi, x_lo) then 8-byte
// (FP64 z; FP32-compensated y_lo, z_lo), so a record takes two aligned
// loads; velocities are 24-byte (FP64) or 12-byte records.
template <int PREC>
struct CState {
    using R = typename State<3, PREC>::R;
    struct __attribute__((aligned(8))) D3 { double a[3]; };
    struct __attribute__((aligned(4))) F3 { float a[3]; };
    __device__ static void load_u(const void *U, uint32_t q, uint32_t ns, R hi[3], R lo[3]) {
        const char *b = static_cast<const char *>(U);
        if constexpr (PREC == 1) {
            const float4 a = *reinterpret_cast<const float4 *>(b + q * 16u);
            const float2 c = *reinterpret_cast<const float2 *>(b + (ns * 16u + q * 8u));
            hi[0] = a.x; hi[1] = a.y; hi[2] = a.z; lo[0] = a.w; lo[1] = c.x; lo[2] = c.y;
        } else {
            const double2 a = *reinterpret_cast<const double2 *>(b + q * 16u);
            hi[0] = a.x; hi[1] = a.y;
            hi[2] = *reinterpret_cast<const double *>(b + (ns * 16u + q * 8u));
            lo[0] = 0.0; lo[1] = 0.0; lo[2] = 0.0;
        }
    }
    __device__ static void store_u(void *U, uint32_t q, uint32_t ns, const R hi[3], const R lo[3]) {
        char *b = static_cast<char *>(U);
        if constexpr (PREC == 1) {
            *reinterpret_cast<float4 *>(b + q * 16u) = make_float4(hi[0], hi[1], hi[2], lo[0]);
            *reinterpret_cast<float2 *>(b + (ns * 16u + q * 8u)) = make_float2(lo[1], lo[2]);
        } else {
            *reinterpret_cast<double2 *>(b + q * 16u) = make_double2(hi[0], hi[1]);
            *reinterpret_cast<double *>(b + (ns * 16u + q * 8u)) = hi[2];
        }
    }
    __device__ static void load_v(const void *V, uint32_t q, R v[3]) {
        if constexpr (PREC == 1) {
            const F3 t = *reinterpret_cast<const F3 *>(static_cast<const char *>(V) + q * 12u);
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = t.a[c];
        } else {
            const D3 t = *reinterpret_cast<const D3 *>(static_cast<const char *>(V) + q * 24u);
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = t.a[c];
        }
    }
    __device__ static void store_v(void *V, uint32_t q, const R v[3]) {
        if constexpr (PREC == 1) {
            F3 t;
#pragma unroll
            for (int c = 0; c < 3; ++c) t.a[c] = v[c];
            *reinterpret_cast<F3 *>(static_cast<char *>(V) + q * 12u) = t;
        } else {
            D3 t;
#pragma unroll
            for (int c = 0; c < 3; ++c) t.a[c] = v[c];
            *reinterpret_cast<D3 *>(static_cast<char *>(V) + q * 24u) = t;
        }
    }
};
template <int PREC>
struct CStore {
    using R = typename State<3, PREC>::R;
    uint32_t q, ns;
    __device__ void u(void *U, const R *hi, const R *lo) const { CState<PREC>::store_u(U, q, ns, hi, lo); }
    __device__ void v(void *V, const R *w) const { CState<PREC>::store_v(V, q, w); }
};

// ... or, in the 2D sweeps, by 32-bit byte offsets from the array base
// (the sweeps run lattices and batches of fewer than 2^28 sites, so a
// 16-byte record's offset fits), which the accesses take as base + offset.
template <int PREC>
struct RowStore {
    using R = typename State<2, PREC>::R;
    using V2 = typename std::conditional<PREC == 1, float2, double2>::type;
    uint32_t g;  // site index
    __device__ void u(void *U, const R *hi, const R *lo) const {
        char *b = static_cast<char *>(U) + g * 16u;
        if constexpr (PREC == 1) *reinterpret_cast<float4 *>(b) = make_float4(hi[0], hi[1], lo[0], lo[1]);
        else *reinterpret_cast<double2 *>(b) = make_double2(hi[0], hi[1]);
    }
    __device__ void v(void *V, const R *w) const {
        char *b = static_cast<char *>(V) + g * uint32_t(sizeof(V2));
        *reinterpret_cast<V2 *>(b) = V2{w[0], w[1]};
    }
};

template <int DIM, int PREC, int MODE, class ST>
__device__ inline void integrate_site(const StepParams &P, const ST &st, uint8_t fp, double mass,
                                      typename State<DIM, PREC>::R inv_mass,
                                      typename State<DIM, PREC>::R *uph,
                                      typename State<DIM, PREC>::R *upl,
                                      const typename State<DIM, PREC>::R *F,
                                      typename State<DIM, PREC>::R *w, double *red) {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    if (flag_grip(fp) != 0) {
        // clamped: displacement carried over, velocity stays zero
        if constexpr (MODE != kEnd) st.u(P.u_out, uph, upl);
        if constexpr (MODE == kEnd) {
            R z[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) z[c] = R(0);
            st.v(P.acc, z);
        }
        return;
    }
    const R h = R(0.5 * P.dt);
    const R dt = R(P.dt);
    const R gam = R(P.gamma);
    R acc[DIM];
    site_acc<DIM, PREC>(F, w, mass, inv_mass, gam, acc);
    if constexpr (MODE == kStart) {
        // w holds the full-step velocity at the increment
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            w[c] = w[c] + h * acc[c];
            comp_add(uph[c], upl[c], dt * w[c]);
        }
        st.u(P.u_out, uph, upl);
        st.v(P.v, w);
    } else if constexpr (MODE == kMid) {
        mid_kick_drift<DIM, PREC>(uph, upl, w, acc, h, dt);
        st.u(P.u_out, uph, upl);
        st.v(P.v, w);
    } else if constexpr (MODE == kEnd) {
        // close the step on the full-step velocity
#pragma unroll
        for (int c = 0; c < DIM; ++c) w[c] = w[c] + h * acc[c];
        st.v(P.v, w);
        st.v(P.acc, acc);
        const double mm = mass;
#pragma unroll
        for (int aa = 0; aa < DIM; ++aa) {
#pragma unroll
            for (int bb = 0; bb < DIM; ++bb) red[9 + aa * 3 + bb] += mm * double(w[aa]) * double(w[bb]);
            red[19] += 0.5 * mm * double(w[aa]) * double(w[aa]);
        }
    }
}

// Spring p -> q in direction d from the displacements of both ends: the
// vector and squared length, the critical-stretch test (Eq. 1-2, strict
// r > rc, FP64 where FP32 cannot decide) and the margin of a break.
template <int DIM, int PREC>
struct SpringEval {
    using R = typename State<DIM, PREC>::R;
    R dv[DIM];
    R r2;
    bool brk;
    bool have64;     // d64 / r64 hold the FP64 vector and length
    double margin;
    double e64[DIM];
    double d64[DIM];
    double r64;
};

// (alat: the lattice constant P.a, passed by kernels that keep it in a
// register across their unrolled spring loops)
template <int DIM, int PREC>
__device__ __attribute__((always_inline)) inline void spring_eval(
    const StepParams &P, double alat, const typename TT<PREC>::type &T, int ti, int d,
    const typename State<DIM, PREC>::R *uph, const typename State<DIM, PREC>::R *upl,
    const typename State<DIM, PREC>::R *uqh, const typename State<DIM, PREC>::R *uql, SpringEval<DIM, PREC> &o) {
    using R = typename State<DIM, PREC>::R;
    using G = Geo<DIM>;
    const R a = R(alat);
    const R hy = R(kHalfSqrt3 * alat);
    // lattice vector X0_q - X0_p
    R e[DIM];
    if constexpr (DIM == 2) {
        e[0] = R(G::ex(d)) * a;
        e[1] = R(G::ey(d)) * hy;
        o.e64[0] = G::ex(d) * alat;
        o.e64[1] = G::ey(d) * (kHalfSqrt3 * alat);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            e[c] = R(G::off(d, c)) * a;
            o.e64[c] = double(G::off(d, c)) * alat;
        }
    }
    o.r2 = R(0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        if constexpr (DIM == 3) {
            // 3D: no term for a zero lattice offset, and no low words in
            // FP64 (they are zero); the same values up to the sign of a zero
            const R du = PREC == 1 ? (uqh[c] - uph[c]) + (uql[c] - upl[c]) : uqh[c] - uph[c];
            o.dv[c] = G::off(d, c) == 0 ? du : e[c] + du;
        } else {
            o.dv[c] = e[c] + ((uqh[c] - uph[c]) + (uql[c] - upl[c]));
        }
        o.r2 += o.dv[c] * o.dv[c];
    }
    o.margin = 0.0;
    o.r64 = 0.0;
    o.have64 = false;
    if constexpr (PREC == 1) {
        // FP32 test; inside the band (or above rc) the FP64 test decides
        if (o.r2 > T.z) {
            double s2 = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                o.d64[c] = o.e64[c] + ((double(uqh[c]) - double(uph[c])) + (double(uql[c]) - double(upl[c])));
                s2 += o.d64[c] * o.d64[c];
            }
            o.r64 = sqrt(s2);
            o.have64 = true;
            const double rc = P.types[ti].rc64;
            o.brk = o.r64 > rc;
            o.margin = (o.r64 - rc) / rc;
        } else {
            o.brk = false;
        }
    } else if constexpr (DIM == 3) {
        // FP64, 3D: r^2 against rc^2 (the decision r > rc, except within an
        // ulp of rc^2); the length only for a break's margin
        o.brk = o.r2 > T.w;
        if (o.brk) {
            o.r64 = sqrt(double(o.r2));
            o.margin = (o.r64 - T.z) / T.z;
        }
    } else {
        o.r64 = sqrt(double(o.r2));
        o.have64 = true;
        o.brk = o.r64 > T.z;
        if (o.brk) o.margin = (o.r64 - T.z) / T.z;
    }
}

template <int DIM, int PREC>
__device__ __attribute__((always_inline)) inline void spring_eval(
    const StepParams &P, const typename TT<PREC>::type &T, int ti, int d, const typename State<DIM, PREC>::R *uph,
    const typename State<DIM, PREC>::R *upl, const typename State<DIM, PREC>::R *uqh,
    const typename State<DIM, PREC>::R *uql, SpringEval<DIM, PREC> &o) {
    spring_eval<DIM, PREC>(P, P.a, T, ti, d, uph, upl, uqh, uql, o);
}

// Eq. 2 force of an intact spring added to the force on p.  cubic != 0
// scales it by 1 + c d^2 / r0^2 (d = r - r0), the cubic spring law.
template <int DIM, int PREC>
__device__ __attribute__((always_inline)) inline void spring_force_add(const typename TT<PREC>::type &T,
                                                                       SpringEval<DIM, PREC> &o,
                                                                       typename State<DIM, PREC>::R *F,
                                                                       double cubic = 0.0) {
    if constexpr (PREC == 1) {
        const float rinv = __builtin_amdgcn_rsqf(o.r2);  // r2 is a normal number
        float coef = fmaf(-T.y, rinv, T.x);              // k (r - r0) / r
        if (cubic != 0.0) {
            const float dr = (o.r2 * rinv - T.w) / T.w;   // (r - r0) / r0
            coef *= fmaf(float(cubic) * dr, dr, 1.0f);
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) F[c] = fmaf(coef, o.dv[c], F[c]);
    } else if constexpr (DIM == 3) {
        // k (r - r0) / r = k - k r0 / r from 1 / r
        const double rinv = rsqrt_pos(double(o.r2));
        double coef = fma(-(T.x * T.y), rinv, T.x);
        if (cubic != 0.0) {
            const double dr = (double(o.r2) * rinv - T.y) / T.y;
            coef *= fma(cubic * dr, dr, 1.0);
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) F[c] += coef * o.dv[c];
    } else {
        double coef = T.x * (o.r64 - T.y) / o.r64;
        if (cubic != 0.0) {
            const double dr = (o.r64 - T.y) / T.y;
            coef *= fma(cubic * dr, dr, 1.0);
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            F[c] += coef * o.dv[c];
            o.d64[c] = o.dv[c];
        }
    }
}

// The 3D FP64 force of spring_force_add with -(k r0) precomputed (nkr0 =
// -(T.x * T.y), the same product): the same result.
__device__ __attribute__((always_inline)) inline void spring_force_add_f64(const D4 &T, double nkr0,
                                                                          const SpringEval<3, 0> &o, double *F,
                                                                          double cubic) {
    const double rinv = rsqrt_pos(o.r2);
    double coef = fma(nkr0, rinv, T.x);
    if (cubic != 0.0) {
        const double dr = (double(o.r2) * rinv - T.y) / T.y;
        coef *= fma(cubic * dr, dr, 1.0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] += coef * o.dv[c];
}

// ------------------------------------------------------------ step kernel
// One time step of one site: all incident springs in direction order
// (break test, Eq. 1-2 force), then the integrator.  Everything is read and
// written through P, so a caller may point the state arrays at LDS.  LAW:
// the spring law (LSM_SPRING_*), or -1 to take it from P at run time.
template <int DIM, int PREC, int MODE, int LAW = -1>
__device__ __attribute__((always_inline)) inline void step_site(
    const StepParams &P, const typename TT<PREC>::type *tt, const double *mass_s,
    const typename State<DIM, PREC>::R *imass_s, int g, int i, int j, int k, uint8_t fp, double *red,
    int step_local) {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    using G = Geo<DIM>;
    using Mask = typename G::Mask;
    using TTy = typename TT<PREC>::type;
    const int law = LAW < 0 ? int(P.law) : LAW;
    R uph[DIM], upl[DIM];
    S::load_u(P.u_in, g, P.nsites, uph, upl);
    const Mask mask = reinterpret_cast<const Mask *>(P.mask)[g];
    Mask newmask = mask;
    const int pa = flag_phase(fp);
    const bool commit = (MODE != kEval) || P.commit;
    R F[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) F[c] = R(0);
    int rank = 0;
    // neighbours in groups of kGrp: all loads of a group are issued
    // unconditionally (from the site itself when the neighbour is outside
    // the lattice) before any of them is used
    constexpr int kGrp = 6;
#pragma unroll
    for (int d0 = 0; d0 < G::ND; d0 += kGrp) {
    int qs[kGrp];
    bool inb[kGrp];
    uint8_t fqs[kGrp];
    R uqhs[kGrp][DIM], uqls[kGrp][DIM];
#pragma unroll
    for (int t = 0; t < kGrp; ++t) {
        const int d = d0 + t;
        const int ddi = G::di(d, j & 1), ddj = G::dj(d), ddk = G::dk(d);
        const int qi = i + ddi, qj = j + ddj, qk = k + ddk;
        inb[t] = !(qi < 0 || qi >= P.nx || qj < 0 || qj >= P.ny || qk < 0 || qk >= P.nz);
        qs[t] = inb[t] ? g + ddi + P.nx * (ddj + P.ny * ddk) : g;
        fqs[t] = P.flags[qs[t]];
        S::load_u(P.u_in, qs[t], P.nsites, uqhs[t], uqls[t]);
    }
#pragma unroll
    for (int t = 0; t < kGrp; ++t) {
        const int d = d0 + t;
        if (!inb[t]) continue;
        const uint8_t fq = fqs[t];
        if (fq == kVoid) continue;
        const bool fwd = d < G::NF;
        const int myrank = rank;
        if (fwd) ++rank;
        // a broken spring acts only under the recoverable law, in compression
        const bool was_broken = mask & (Mask(1) << d);
        if (was_broken && law != LSM_SPRING_RECOVER) continue;
        const R *uqh = uqhs[t];
        const R *uql = uqls[t];
        const int pb = flag_phase(fq);
        const int ti = G::geom(d) * (LSM_MAX_PHASES * LSM_MAX_PHASES) + pa * LSM_MAX_PHASES + pb;
        const TTy T = tt[ti];
        SpringEval<DIM, PREC> o;
        spring_eval<DIM, PREC>(P, T, ti, d, uph, upl, uqh, uql, o);
        if (was_broken) {
            const double r0 = P.types[ti].r0_64;
            if (!(double(o.r2) < r0 * r0)) continue;
            o.brk = false;
        }
        const bool brk = o.brk;
        const double margin = o.margin;
        double *d64 = o.d64;
        double &r64 = o.r64;
        const R *dv = o.dv;
        const double *e64 = o.e64;
        if (brk) {
            if (commit) {
                newmask |= Mask(1) << d;
                if (fwd) {
                    const uint32_t idx = event_slot(P.ctl);
                    if (idx < P.ev_cap) {
                        lsm_event ev;
                        ev.increment = P.ctl->inc;
                        ev.step = P.ctl->step_base + step_local;
                        ev.spring_id = int64_t(P.sbase[g]) + myrank;
                        ev.margin = margin;
                        P.events[idx] = ev;
                    }
                }
            }
            continue;
        }
        spring_force_add<DIM, PREC>(T, o, F, law == LSM_SPRING_CUBIC ? P.law_c : 0.0);
        if constexpr (MODE == kEnd) {
            if (fwd) {
                // virial (Eq. 7) and potential energy (Eq. 1) in FP64
                const TypeRec &T64 = P.types[ti];
                if (!o.have64) {
                    double s2 = 0.0;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        d64[c] = e64[c] + ((double(uqh[c]) - double(uph[c])) +
                                           (double(uql[c]) - double(upl[c])));
                        s2 += d64[c] * d64[c];
                    }
                    r64 = sqrt(s2);
                }
                double coef64 = T64.k64 * (r64 - T64.r0_64) / r64;
                const double dl = r64 - T64.r0_64;
                double pe = 0.5 * T64.k64 * dl * dl;
                if (law == LSM_SPRING_CUBIC) {
                    const double dr = dl / T64.r0_64;
                    coef64 *= 1.0 + P.law_c * dr * dr;
                    pe += 0.25 * T64.k64 * P.law_c * dl * dl * dr * dr;
                }
#pragma unroll
                for (int aa = 0; aa < DIM; ++aa)
#pragma unroll
                    for (int bb = 0; bb < DIM; ++bb) red[aa * 3 + bb] += d64[aa] * (coef64 * d64[bb]);
                red[18] += pe;
            }
        }
    }
    }
    if (commit && newmask != mask) reinterpret_cast<Mask *>(P.mask)[g] = newmask;

    if constexpr (MODE == kEval) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) P.f64[int64_t(g) * DIM + c] = double(F[c]);
    } else {
        R w[DIM];
        if (flag_grip(fp) == 0) S::load_v(P.v, g, P.nsites, w);
        integrate_site<DIM, PREC, MODE>(P, SiteStore<DIM, PREC>{g, P.nsites}, fp, mass_s[pa], imass_s[pa],
                                        uph, upl, F, w, red);
    }
}

template <int DIM, int PREC, int MODE>
__global__ __launch_bounds__(kBlock) void k_step(StepParams P, int step_local) {
    using R = typename State<DIM, PREC>::R;
    using TTy = typename TT<PREC>::type;

    __shared__ TTy tt[kMaxTypes];
    __shared__ double mass_s[LSM_MAX_PHASES];
    __shared__ R imass_s[LSM_MAX_PHASES];  // R(1 / m), once per workgroup
    __shared__ double red_lds[MODE == kEnd ? kNumPartials : 1][kBlock / 64];
    for (int t = threadIdx.x; t < kMaxTypes; t += kBlock) tt[t] = TT<PREC>::make(P.types[t]);
    if (threadIdx.x < LSM_MAX_PHASES) {
        mass_s[threadIdx.x] = P.mass[threadIdx.x];
        imass_s[threadIdx.x] = R(1.0 / P.mass[threadIdx.x]);
    }
    __syncthreads();

    int i, j, k;
    bool active;
    if (P.plist) {
        // one thread per particle; each XCD takes a contiguous run of
        // workgroups (particles of neighbouring rows and planes share its L2)
        const int b = blockIdx.x;
        const int lb = (b & 7) * (P.c_blocks >> 3) + (b >> 3);
        const int64_t t = int64_t(lb) * kBlock + threadIdx.x;
        active = t < P.n_part;
        const uint32_t pc = active ? P.plist[t] : 0u;
        i = int(pc & 1023u);
        j = int((pc >> 10) & 2047u);
        k = int(pc >> 21);
    } else {
        tile_coords(P, i, j, k, active);
    }
    const int g = active ? i + P.nx * (j + P.ny * k) : 0;
    const uint8_t fp = active ? P.flags[g] : kVoid;
    active = active && fp != kVoid;

    double red[MODE == kEnd ? kNumPartials : 1];
#pragma unroll
    for (int v = 0; v < (MODE == kEnd ? kNumPartials : 1); ++v) red[v] = 0.0;

    if (active) step_site<DIM, PREC, MODE>(P, tt, mass_s, imass_s, g, i, j, k, fp, red, step_local);

    if constexpr (MODE == kEnd) {
        block_sum(red, red_lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int v = 0; v < kNumPartials; ++v) P.partials[int64_t(blockIdx.x) * kNumPartials + v] = red[v];
        }
    }
}

// wave_shl:1 -> lane l reads lane l + 1; wave_shr:1 -> lane l reads lane l - 1
// (the edge lane reads zero; edge lanes are never owned).
__device__ inline int lane_next(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true); }
__device__ inline int lane_prev(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true); }
__device__ inline float lane_next(float x) { return __int_as_float(lane_next(__float_as_int(x))); }
__device__ inline float lane_prev(float x) { return __int_as_float(lane_prev(__float_as_int(x))); }
__device__ inline double lane_next(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = lane_next(int(b & 0xFFFFFFFFll)), hi = lane_next(int(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ inline double lane_prev(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = lane_prev(int(b & 0xFFFFFFFFll)), hi = lane_prev(int(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Calls f(std::integral_constant<int, t>) for t = T .. N - 1 in order, so
// each unrolled row can use t in template arguments.
// Interior step of a 3D lattice in the compact layout: one thread per
// particle (raster order, which is the canonical particle order), state,
// flags and break bits stored per particle, so a wavefront's loads and
// stores touch only solid sites.  The 18 neighbours lie in 9 grid rows
// (x-lines); one entry of the row table per row -- the particle index of
// the row's site at the particle's x, whether that site is solid, and the
// phases of it and its two x-neighbours -- gives the indices and phases of
// the neighbours in that row (raster order makes a row's solid sites
// consecutive particles); the own row's neighbours p - 1 and p + 1 are the
// adjacent lanes.  (Taking the other rows' x +- 1 neighbours from the
// adjacent lanes' same-x neighbours as well, with a row-grouped summation
// order, measured slower: 323 against 285 us per C3 FP64 step.)  Every
// load of a particle is issued before
// any of its stores; the events of forward springs that break are logged
// after all loads (the test is redone for the margin), before the update.
// Arithmetic and summation order are the gather kernel's, so state, break
// bits and events are bitwise the same.
template <int PREC, bool ROW32>
__global__ __launch_bounds__(kBlock) void k_step_c3(StepParams P, int step_local) {
    constexpr int GRP = 6;  // neighbour loads per group (9 or 18, or the next group's loads in
                            // flight during the current one, measured slower)
    using CS = CState<PREC>;
    using R = typename CS::R;
    using G = Geo<3>;
    using TTy = typename TT<PREC>::type;
    constexpr int NG = G::ND / GRP;
    static_assert(G::ND % GRP == 0, "groups must tile the 18 directions");
    __shared__ TTy tt[kMaxTypes];
    __shared__ double mass_s[LSM_MAX_PHASES];
    __shared__ R imass_s[LSM_MAX_PHASES];
    for (int t = threadIdx.x; t < kMaxTypes; t += kBlock) tt[t] = TT<PREC>::make(P.types[t]);
    if (threadIdx.x < LSM_MAX_PHASES) {
        mass_s[threadIdx.x] = P.mass[threadIdx.x];
        imass_s[threadIdx.x] = R(1.0 / P.mass[threadIdx.x]);
    }
    __syncthreads();
    const int b = blockIdx.x;
    const int lb = (b & 7) * (P.c_blocks >> 3) + (b >> 3);
    const int p = lb * kBlock + int(threadIdx.x);
    const int lane = int(threadIdx.x) & 63;
    if (p >= P.n_part) return;
    const uint32_t pc = P.plist[p];
    const int i = int(pc & 1023u), j = int((pc >> 10) & 2047u), k = int(pc >> 21);
    const int gg = i + P.nx * (j + P.ny * k);
    const uint32_t ns = uint32_t(P.nsites);
    R uph[3], upl[3], w[3];
    CS::load_u(P.u_in, uint32_t(p), ns, uph, upl);
    CS::load_v(P.v, uint32_t(p), w);
    const uint32_t mask = reinterpret_cast<const uint32_t *>(P.mask)[p];
    const uint8_t fp = P.flags[p];
    // row entries: slot (dj + 1) * 3 + (dk + 1); a row off the grid reads
    // the particle's own entry (all its springs there are absent).  ROW32:
    // single-phase lattices keep (particles before << 1) | solid in 32 bits.
    uint64_t row[9];
#pragma unroll
    for (int sl = 0; sl < 9; ++sl) {
        if (sl == 4) continue;  // own row: p - 1 and p + 1
        const int dj = sl / 3 - 1, dk = sl % 3 - 1;
        const bool in = j + dj >= 0 && j + dj < P.ny && k + dk >= 0 && k + dk < P.nz;
        const uint32_t gq = uint32_t(in ? gg + P.nx * (dj + P.ny * dk) : gg);
        if constexpr (ROW32) {
            const uint32_t e = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(P.crow) + gq * 4u);
            row[sl] = (uint64_t(e >> 1) << 32) | (uint64_t(e & 1u) << 12);
        } else {
            row[sl] = *reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(P.crow) + gq * 8u);
        }
    }
    if constexpr (ROW32) row[4] = 0;
    else row[4] = *reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(P.crow) + uint32_t(gg) * 8u);
    const uint32_t qmax = uint32_t(P.n_part - 1);
    // neighbour in direction d: index (clamped, for absent springs) and phase
    auto nbr = [&](int d, uint32_t &q, int &pb) {
        const int dx = G::di(d, 0), sl = (G::dj(d) + 1) * 3 + (G::dk(d) + 1);
        const uint64_t e = row[sl];
        pb = int((e >> (4 * (dx + 1))) & 15u);
        if (sl == 4) {
            q = uint32_t(p + dx);
        } else {
            const uint32_t r = uint32_t(e >> 32);
            q = dx < 0 ? r - 1u : (dx > 0 ? r + uint32_t((e >> 12) & 1u) : r);
        }
        q = min(q, qmax);
    };
    // the x-neighbours p - 1 and p + 1 are the adjacent lanes (particles are
    // consecutive across a wavefront): their displacements come by DPP, and
    // only the edge lanes load them
    auto xnbr = [&](int dx, R *qh, R *ql) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            qh[c] = dx > 0 ? lane_next(uph[c]) : lane_prev(uph[c]);
            ql[c] = dx > 0 ? lane_next(upl[c]) : lane_prev(upl[c]);
        }
        if (lane == (dx > 0 ? 63 : 0)) CS::load_u(P.u_in, min(uint32_t(p + dx), qmax), ns, qh, ql);
    };
    const int pa = flag_phase(fp);
    R F[3] = {R(0), R(0), R(0)};
    uint32_t newmask = mask, fbrk = 0;
    R uqh[GRP][3], uql[GRP][3];
    int pbs[GRP];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
#pragma unroll
        for (int t = 0; t < GRP; ++t) {
            const int d = gi * GRP + t;
            uint32_t q;
            nbr(d, q, pbs[t]);
            if (G::dj(d) == 0 && G::dk(d) == 0) xnbr(G::di(d, 0), uqh[t], uql[t]);
            else CS::load_u(P.u_in, q, ns, uqh[t], uql[t]);
        }
#pragma unroll
        for (int t = 0; t < GRP; ++t) {
            const int d = gi * GRP + t;
            if (mask & (1u << d)) continue;
            const int ti = G::geom(d) * (LSM_MAX_PHASES * LSM_MAX_PHASES) + pa * LSM_MAX_PHASES + pbs[t];
            const TTy T = tt[ti];
            SpringEval<3, PREC> o;
            spring_eval<3, PREC>(P, T, ti, d, uph, upl, uqh[t], uql[t], o);
            if (o.brk) {
                newmask |= 1u << d;
                if (d < G::NF) fbrk |= 1u << d;
                continue;
            }
            spring_force_add<3, PREC>(T, o, F);
        }
    }
    // (before the update, which advances uph / upl in place)
    while (fbrk) {
        const int d = __builtin_ctz(fbrk);
        fbrk &= fbrk - 1u;
        uint32_t q;
        int pb;
        nbr(d, q, pb);
        R qh[3], ql[3];
        CS::load_u(P.u_in, q, ns, qh, ql);
        const int ti = G::geom(d) * (LSM_MAX_PHASES * LSM_MAX_PHASES) + pa * LSM_MAX_PHASES + pb;
        SpringEval<3, PREC> o;
        spring_eval<3, PREC>(P, tt[ti], ti, d, uph, upl, qh, ql, o);
        const uint32_t idx = event_slot(P.ctl);
        if (idx < P.ev_cap) {
            lsm_event ev;
            ev.increment = P.ctl->inc;
            ev.step = P.ctl->step_base + step_local;
            ev.spring_id = int64_t(P.sbase[gg]) + __popc(~P.cabs[p] & ((1u << d) - 1u));
            ev.margin = o.margin;
            P.events[idx] = ev;
        }
    }
    double red[1] = {0.0};
    integrate_site<3, PREC, kMid>(P, CStore<PREC>{uint32_t(p), ns}, fp, mass_s[pa], imass_s[pa], uph, upl, F, w,
                                  red);
    if (newmask != mask) reinterpret_cast<uint32_t *>(P.mask)[p] = newmask;
}

// Interior step of a single-phase 3D lattice in the compact layout, with
// the displacements a workgroup reads staged in LDS.  The workgroup's
// kC3WinBlock consecutive particles lie between grid sites g0 and g1; all their
// neighbours in plane offset dk lie between sites g0 - nx - 1 and
// g1 + nx + 1 of that plane, a contiguous run of particles (raster order),
// the window of dk.  The three windows are copied one after the other into
// an LDS pool of POOL records with coalesced loads before any spring is
// evaluated.  A per-particle entry per off-row grid row -- the offset in
// that plane's window of the row's site at the particle's x, and whether
// that site is solid -- gives the neighbours in the row (x - 1: entry - 1,
// x: entry, x + 1: entry + solid bit); the own row's neighbours are p - 1
// and p + 1.  A workgroup whose windows exceed the pool reads every
// neighbour from global memory.  LAW is the spring law (LSM_SPRING_*: a
// broken spring acts again in compression under the recoverable law, the
// cubic law scales the force).  Arithmetic and summation order are those
// of the gather kernel, so state, break bits and events are bitwise the
// same.
template <int PREC, int POOL, int LAW>
__global__ __launch_bounds__(kC3WinBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_step_c3w(StepParams P,
                                                                                             int step_local) {
    constexpr int GRP = PREC ? 3 : 6;  // FP32-compensated: fewer registers, four waves per SIMD
    using CS = CState<PREC>;
    using R = typename CS::R;
    using G = Geo<3>;
    using TTy = typename TT<PREC>::type;
    using VA = typename std::conditional<PREC == 1, float4, double2>::type;  // 16-byte record part
    using VB = typename std::conditional<PREC == 1, float2, double>::type;   // 8-byte record part
    constexpr int NG = G::ND / GRP;
    constexpr int NIT = (POOL + kC3WinBlock - 1) / kC3WinBlock;
    static_assert(G::ND % GRP == 0, "groups must tile the 18 directions");
    // pool slot x + 1 holds staged record x: every offset the row entries
    // give, -1 .. window length, lands inside (slots 0 .. POOL + 1)
    __shared__ VA wa[POOL + 2];
    __shared__ VB wb[POOL + 2];
    const int b = blockIdx.x;
    const int lb = (b & 7) * (P.c_wblocks >> 3) + (b >> 3);
    if (lb * kC3WinBlock >= P.n_part) return;  // the whole workgroup
    const int p = lb * kC3WinBlock + int(threadIdx.x);
    const bool act = p < P.n_part;
    const uint32_t pp = uint32_t(act ? p : P.n_part - 1);
    const uint32_t ns = uint32_t(P.nsites);
    const char *ub = static_cast<const char *>(P.u_in);
    // windows: first particle, records staged, pool offset (uniform)
    const uint32_t wb0 = P.cwin[lb * 8 + 0], wb1 = P.cwin[lb * 8 + 1], wb2 = P.cwin[lb * 8 + 2];
    const uint32_t wl0 = P.cwin[lb * 8 + 3], wl1 = P.cwin[lb * 8 + 4], wl2 = P.cwin[lb * 8 + 5];
    const uint32_t nst = wl0 + wl1 + wl2;  // >= 1: the own particles are in window 1
    const bool fit = nst <= uint32_t(POOL);
    // own state first, so its loads are in flight during the window copy
    R w[3];
    CS::load_v(P.v, pp, w);
    const uint32_t mask = reinterpret_cast<const uint32_t *>(P.mask)[pp];
    const uint8_t fp = P.flags[pp];
    const uint4 er = reinterpret_cast<const uint4 *>(P.crel)[pp];
    // absent springs (void or off-grid neighbour): the recoverable law tells
    // them from broken ones
    const uint32_t absent = LAW == LSM_SPRING_RECOVER ? P.cabs[pp] : 0u;
    // window copy: the loads of every round the windows need (index clamped
    // to the last record), then the stores.  (Batches of three or four
    // rounds measured 1-3 % slower; loads straight into LDS, 249 against
    // 228 us per C3 FP64 step.)
    struct Rec {
        VA a;
        VB b;
    };
    auto fetch = [&](int it) {
        const uint32_t x = min(threadIdx.x + uint32_t(it * kC3WinBlock), nst - 1u);
        const uint32_t q = x + (x < wl0 ? wb0 : (x < wl0 + wl1 ? wb1 - wl0 : wb2 - wl0 - wl1));
        return Rec{*reinterpret_cast<const VA *>(ub + q * 16u), *reinterpret_cast<const VB *>(ub + (ns * 16u + q * 8u))};
    };
    auto put = [&](int it, const Rec &r) {
        const uint32_t x = threadIdx.x + uint32_t(it * kC3WinBlock);
        if (x < nst) {
            wa[x + 1] = r.a;
            wb[x + 1] = r.b;
        }
    };
    if (fit) {
        const int nr = int((nst + kC3WinBlock - 1) / kC3WinBlock);  // rounds needed (uniform)
        Rec r[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it)
            if (it < nr) r[it] = fetch(it);
#pragma unroll
        for (int it = 0; it < NIT; ++it)
            if (it < nr) put(it, r[it]);
    }
    __syncthreads();
    if (!act) return;
    const uint32_t qmax = uint32_t(P.n_part - 1);
    const uint32_t wbase[3] = {wb0, wb1, wb2};
    const uint32_t soff[3] = {1u, 1u + wl0, 1u + wl0 + wl1};  // slot of each window's first record
    // spring types of the two geometry classes (phase 0 with itself)
    const TTy T0 = TT<PREC>::make(P.types[0]), T1 = TT<PREC>::make(P.types[LSM_MAX_PHASES * LSM_MAX_PHASES]);
    const double nk0 = -(double(T0.x) * double(T0.y)), nk1 = -(double(T1.x) * double(T1.y));  // FP64 only
    const double alat = P.a;
    const double cubic = LAW == LSM_SPRING_CUBIC ? P.law_c : 0.0;
    const double mass = P.mass[0];
    const R imass = R(1.0 / mass);
    auto lds = [&](uint32_t x, R *qh, R *ql) {
        const VA a = wa[x];
        const VB c = wb[x];
        if constexpr (PREC == 1) {
            qh[0] = a.x; qh[1] = a.y; qh[2] = a.z; ql[0] = a.w; ql[1] = c.x; ql[2] = c.y;
        } else {
            qh[0] = a.x; qh[1] = a.y; qh[2] = c;
            ql[0] = 0.0; ql[1] = 0.0; ql[2] = 0.0;
        }
    };
    // record t of window wi: from the pool (an offset outside the window,
    // -1 or the window length, belongs to an absent spring and reads a
    // slot of another window or a spare one), or from global memory when
    // the windows exceed the pool
    auto ld = [&](auto fit_c, int wi, uint32_t t, R *qh, R *ql) {
        if constexpr (decltype(fit_c)::value) lds(soff[wi] + t, qh, ql);
        else CS::load_u(P.u_in, min(wbase[wi] + t, qmax), ns, qh, ql);
    };
    const uint32_t t0 = uint32_t(p) - wb1;
    // entries of the off-row rows, slot (dj + 1) * 3 + (dk + 1) without the own row
    const uint32_t ent[8] = {er.x & 0xFFFFu, er.x >> 16, er.y & 0xFFFFu, er.y >> 16,
                             er.z & 0xFFFFu, er.z >> 16, er.w & 0xFFFFu, er.w >> 16};
    // neighbour in direction d: window and offset in it
    auto nbr = [&](int d, int &wi, uint32_t &t) {
        const int dx = G::di(d, 0), sl = (G::dj(d) + 1) * 3 + (G::dk(d) + 1);
        wi = G::dk(d) + 1;
        if (sl == 4) {
            t = t0 + uint32_t(dx);
        } else {
            const uint32_t e = ent[sl < 4 ? sl : sl - 1];
            const uint32_t r = e >> 1;
            t = dx < 0 ? r - 1u : (dx > 0 ? r + (e & 1u) : r);
        }
    };
    auto body = [&](auto fit_c) {
        R uph[3], upl[3];
        ld(fit_c, 1, t0, uph, upl);
        R F[3] = {R(0), R(0), R(0)};
        uint32_t newmask = mask, fbrk = 0;
        R uqh[GRP][3], uql[GRP][3];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
#pragma unroll
            for (int t = 0; t < GRP; ++t) {
                int wi;
                uint32_t tq;
                nbr(gi * GRP + t, wi, tq);
                ld(fit_c, wi, tq, uqh[t], uql[t]);
            }
#pragma unroll
            for (int t = 0; t < GRP; ++t) {
                const int d = gi * GRP + t;
                // a broken spring acts only under the recoverable law, in compression
                if (((LAW == LSM_SPRING_RECOVER ? absent : mask) >> d) & 1u) continue;
                const int ti = G::geom(d) * (LSM_MAX_PHASES * LSM_MAX_PHASES);
                const TTy T = G::geom(d) ? T1 : T0;
                SpringEval<3, PREC> o;
                spring_eval<3, PREC>(P, alat, T, ti, d, uph, upl, uqh[t], uql[t], o);
                if constexpr (LAW == LSM_SPRING_RECOVER) {
                    if ((mask >> d) & 1u) {
                        const double r0 = P.types[ti].r0_64;
                        if (!(double(o.r2) < r0 * r0)) continue;
                        o.brk = false;
                    }
                }
                if (o.brk) {
                    newmask |= 1u << d;
                    if (d < G::NF) fbrk |= 1u << d;
                    continue;
                }
                if constexpr (PREC == 0) spring_force_add_f64(T, G::geom(d) ? nk1 : nk0, o, F, cubic);
                else spring_force_add<3, PREC>(T, o, F, cubic);
            }
        }
        // events of forward springs that break (before the update, which
        // advances uph / upl in place)
        if (fbrk) {
            const uint32_t pc = P.plist[p];
            const int i = int(pc & 1023u), j = int((pc >> 10) & 2047u), k = int(pc >> 21);
            const int gg = i + P.nx * (j + P.ny * k);
            // (directions unrolled: the row entries and windows stay in registers)
#pragma unroll
            for (int d = 0; d < G::NF; ++d) {
                if (!(fbrk & (1u << d))) continue;
                int wi;
                uint32_t tq;
                nbr(d, wi, tq);
                R qh[3], ql[3];
                ld(fit_c, wi, tq, qh, ql);
                const int ti = G::geom(d) * (LSM_MAX_PHASES * LSM_MAX_PHASES);
                SpringEval<3, PREC> o;
                spring_eval<3, PREC>(P, alat, G::geom(d) ? T1 : T0, ti, d, uph, upl, qh, ql, o);
                const uint32_t idx = event_slot(P.ctl);
                if (idx < P.ev_cap) {
                    lsm_event ev;
                    ev.increment = P.ctl->inc;
                    ev.step = P.ctl->step_base + step_local;
                    ev.spring_id = int64_t(P.sbase[gg]) + __popc(~P.cabs[p] & ((1u << d) - 1u));
                    ev.margin = o.margin;
                    P.events[idx] = ev;
                }
            }
        }
        double red[1] = {0.0};
        integrate_site<3, PREC, kMid>(P, CStore<PREC>{uint32_t(p), ns}, fp, mass, imass, uph, upl, F, w, red);
        if (newmask != mask) reinterpret_cast<uint32_t *>(P.mask)[p] = newmask;
    };
    if (fit) body(std::true_type{});
    else body(std::false_type{});
}

// ------------------------------------------------------- local fields
// Local stress and strain of the current state (Section 3.1: the virial
// stress of Eq. 7 over a neighbourhood and the Lagrangian strain of the
// field figure).  One thread per particle p (site site_of[p]); FP64 from
// the (hi, lo) displacements.
//
// Virial contribution s^p_ab = 1/2 sum over p's intact springs of
// (x_q - x_p)_a f_b (f the Eq. 2 force on p from q) - m v_a v_b, written to
// out[p] (dim x dim).
template <int DIM, int PREC>
__global__ __launch_bounds__(256) void k_virial(StepParams P, const int32_t *site_of, double *out) {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    using G = Geo<DIM>;
    using Mask = typename G::Mask;
    // (k, r0) of every spring type, staged in LDS: a type read per spring
    // from global memory waits on its own load
    __shared__ double2 tkr[kMaxTypes];
    for (int t = threadIdx.x; t < kMaxTypes; t += 256) tkr[t] = make_double2(P.types[t].k64, P.types[t].r0_64);
    __syncthreads();
    const int p = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (p >= P.n_part) return;
    const int g = site_of[p];
    const int i = g % P.nx, j = (g / P.nx) % P.ny, k = g / (P.nx * P.ny);
    const uint8_t fp = P.flags[g];
    const int pa = flag_phase(fp);
    const Mask mask = reinterpret_cast<const Mask *>(P.mask)[g];
    R uph[DIM], upl[DIM], w[DIM];
    S::load_u(P.u_in, g, P.nsites, uph, upl);
    S::load_v(P.v, g, P.nsites, w);
    double sv[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) sv[a][b] = 0.0;
    // neighbours in groups of six: the flag and displacement loads of a
    // group are issued unconditionally (from the site itself off the
    // lattice) before any of them is used
    constexpr int kGrp = 6;
#pragma unroll
    for (int d0 = 0; d0 < G::ND; d0 += kGrp) {
    bool inb[kGrp];
    uint8_t fqs[kGrp];
    R uqhs[kGrp][DIM], uqls[kGrp][DIM];
#pragma unroll
    for (int t = 0; t < kGrp; ++t) {
        const int d = d0 + t;
        const int ddi = G::di(d, j & 1), ddj = G::dj(d), ddk = G::dk(d);
        const int qi = i + ddi, qj = j + ddj, qk = k + ddk;
        inb[t] = !(qi < 0 || qi >= P.nx || qj < 0 || qj >= P.ny || qk < 0 || qk >= P.nz);
        const int q = inb[t] ? g + ddi + P.nx * (ddj + P.ny * ddk) : g;
        fqs[t] = P.flags[q];
        S::load_u(P.u_in, q, P.nsites, uqhs[t], uqls[t]);
    }
#pragma unroll
    for (int t = 0; t < kGrp; ++t) {
        const int d = d0 + t;
        if (!inb[t]) continue;
        const uint8_t fq = fqs[t];
        const bool was_broken = mask & (Mask(1) << d);
        if (fq == kVoid || (was_broken && P.law != LSM_SPRING_RECOVER)) continue;
        const R *uqh = uqhs[t];
        const R *uql = uqls[t];
        double dd[DIM], r2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double e;
            if constexpr (DIM == 2) e = (c == 0 ? G::ex(d) : G::ey(d) * kHalfSqrt3) * P.a;
            else e = double(G::off(d, c)) * P.a;
            dd[c] = e + ((double(uqh[c]) - double(uph[c])) + (double(uql[c]) - double(upl[c])));
            r2 += dd[c] * dd[c];
        }
        const double2 T = tkr[G::geom(d) * (LSM_MAX_PHASES * LSM_MAX_PHASES) + pa * LSM_MAX_PHASES + flag_phase(fq)];
        const double k64 = T.x, r0 = T.y;
        const double r = sqrt(r2);
        if (was_broken && !(r < r0)) continue;  // recoverable law: compression only
        double coef = k64 * (r - r0) / r;
        if (P.law == LSM_SPRING_CUBIC) {
            const double dr = (r - r0) / r0;
            coef *= 1.0 + P.law_c * dr * dr;
        }
        const double half_coef = 0.5 * coef;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) sv[a][b] += dd[a] * (half_coef * dd[b]);
    }
    }
    const double m = P.mass[pa];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) out[(int64_t(p) * DIM + a) * DIM + b] = sv[a][b] - m * double(w[a]) * double(w[b]);
}

// Virial stress over p's domain: p alone (radius 0) or p and the particles
// it shares a spring with, broken or not (radius 1), per site volume.
template <int DIM>
__global__ __launch_bounds__(256) void k_virial_domain(StepParams P, const int32_t *site_of, const int32_t *part_of,
                                                       const double *s, double *out, int radius, double vsite) {
    using G = Geo<DIM>;
    const int p = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (p >= P.n_part) return;
    double acc[DIM * DIM];
#pragma unroll
    for (int e = 0; e < DIM * DIM; ++e) acc[e] = s[int64_t(p) * DIM * DIM + e];
    int count = 1;
    if (radius > 0) {
        const int g = site_of[p];
        const int i = g % P.nx, j = (g / P.nx) % P.ny, k = g / (P.nx * P.ny);
        // every neighbour's particle index first (-1: void or off the
        // lattice), then their contributions in groups of three, loaded
        // unconditionally (p's own for a missing neighbour) before use
        int qs[G::ND];
#pragma unroll
        for (int d = 0; d < G::ND; ++d) {
            const int ddi = G::di(d, j & 1), ddj = G::dj(d), ddk = G::dk(d);
            const int qi = i + ddi, qj = j + ddj, qk = k + ddk;
            const bool inb = !(qi < 0 || qi >= P.nx || qj < 0 || qj >= P.ny || qk < 0 || qk >= P.nz);
            const int q = part_of[inb ? g + ddi + P.nx * (ddj + P.ny * ddk) : g];
            qs[d] = inb ? q : -1;
        }
        constexpr int kGrp = 3;
#pragma unroll
        for (int d0 = 0; d0 < G::ND; d0 += kGrp) {
            double sq[kGrp][DIM * DIM];
#pragma unroll
            for (int t = 0; t < kGrp; ++t) {
                const int64_t q = qs[d0 + t] >= 0 ? qs[d0 + t] : p;
#pragma unroll
                for (int e = 0; e < DIM * DIM; ++e) sq[t][e] = s[q * DIM * DIM + e];
            }
#pragma unroll
            for (int t = 0; t < kGrp; ++t) {
                if (qs[d0 + t] < 0) continue;
#pragma unroll
                for (int e = 0; e < DIM * DIM; ++e) acc[e] += sq[t][e];
                ++count;
            }
        }
    }
    const double inv = 1.0 / (double(count) * vsite);
#pragma unroll
    for (int e = 0; e < DIM * DIM; ++e) out[int64_t(p) * DIM * DIM + e] = acc[e] * inv;
}

// Lagrangian strain: J = (sum d d0^T)(sum d0 d0^T)^-1 over p's first
// nearest neighbours (2D: the six lattice neighbours; 3D: the six face
// neighbours), broken springs included; eps = (J^T J - I) / 2, NaN where
// the reference vectors do not span the space.
template <int DIM, int PREC>
__global__ __launch_bounds__(256) void k_strain(StepParams P, const int32_t *site_of, double *out) {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    using G = Geo<DIM>;
    const int p = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (p >= P.n_part) return;
    const int g = site_of[p];
    const int i = g % P.nx, j = (g / P.nx) % P.ny, k = g / (P.nx * P.ny);
    R uph[DIM], upl[DIM];
    S::load_u(P.u_in, g, P.nsites, uph, upl);
    double A[DIM][DIM], B[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) A[a][b] = B[a][b] = 0.0;
    // the first nearest neighbours' flags and displacements, loaded
    // unconditionally (the site's own off the lattice) before use
    bool inb[G::ND];
    uint8_t fqs[G::ND];
    R uqhs[G::ND][DIM], uqls[G::ND][DIM];
#pragma unroll
    for (int d = 0; d < G::ND; ++d) {
        if (G::geom(d) != 0) continue;
        const int ddi = G::di(d, j & 1), ddj = G::dj(d), ddk = G::dk(d);
        const int qi = i + ddi, qj = j + ddj, qk = k + ddk;
        inb[d] = !(qi < 0 || qi >= P.nx || qj < 0 || qj >= P.ny || qk < 0 || qk >= P.nz);
        const int q = inb[d] ? g + ddi + P.nx * (ddj + P.ny * ddk) : g;
        fqs[d] = P.flags[q];
        S::load_u(P.u_in, q, P.nsites, uqhs[d], uqls[d]);
    }
#pragma unroll
    for (int d = 0; d < G::ND; ++d) {
        if (G::geom(d) != 0) continue;  // first nearest neighbours only
        if (!inb[d] || fqs[d] == kVoid) continue;
        const R *uqh = uqhs[d];
        const R *uql = uqls[d];
        double d0[DIM], dd[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            if constexpr (DIM == 2) d0[c] = (c == 0 ? G::ex(d) : G::ey(d) * kHalfSqrt3) * P.a;
            else d0[c] = double(G::off(d, c)) * P.a;
            dd[c] = d0[c] + ((double(uqh[c]) - double(uph[c])) + (double(uql[c]) - double(upl[c])));
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                A[a][b] += d0[a] * d0[b];
                B[a][b] += dd[a] * d0[b];
            }
    }
    // inverse of A by its adjugate
    double Ai[DIM][DIM], det, amax = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) amax = fmax(amax, fabs(A[a][b]));
    if constexpr (DIM == 2) {
        det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        Ai[0][0] = A[1][1]; Ai[0][1] = -A[0][1]; Ai[1][0] = -A[1][0]; Ai[1][1] = A[0][0];
    } else {
        Ai[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        Ai[0][1] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
        Ai[0][2] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
        Ai[1][0] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
        Ai[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
        Ai[1][2] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
        Ai[2][0] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
        Ai[2][1] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
        Ai[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        det = A[0][0] * Ai[0][0] + A[0][1] * Ai[1][0] + A[0][2] * Ai[2][0];
    }
    double* o = out + int64_t(p) * DIM * DIM;
    double tiny = 1e-12;
#pragma unroll
    for (int c = 0; c < DIM; ++c) tiny *= amax;
    if (!(fabs(det) > tiny)) {
#pragma unroll
        for (int e = 0; e < DIM * DIM; ++e) o[e] = __longlong_as_double(0x7FF8000000000000LL);
        return;
    }
    double J[DIM][DIM];
    const double inv_det = 1.0 / det;  // one division instead of nine
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) t += B[a][c] * Ai[c][b];
            J[a][b] = t * inv_det;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) t += J[c][a] * J[c][b];
            o[a * DIM + b] = 0.5 * (t - (a == b ? 1.0 : 0.0));
        }
}

// Copies between the site-grid state (displacements u_grid, velocities
// v_grid, break bits m_grid, stride P.nsites) and the compact one; the
// compact break bits also carry the absent-spring bits.
template <int PREC, bool TO_COMPACT>
__global__ __launch_bounds__(256) void k_pack_c3(StepParams P, void *u_grid, void *v_grid, uint32_t *m_grid,
                                                 void *u_c, void *v_c, uint32_t *m_c, uint32_t cn) {
    using S = State<3, PREC>;
    using CS = CState<PREC>;
    using R = typename S::R;
    const int p = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (p >= P.n_part) return;
    const uint32_t pc = P.plist[p];
    const int g = int(pc & 1023u) + P.nx * (int((pc >> 10) & 2047u) + P.ny * int(pc >> 21));
    R hi[3], lo[3], w[3];
    if constexpr (TO_COMPACT) {
        S::load_u(u_grid, g, P.nsites, hi, lo);
        S::load_v(v_grid, g, P.nsites, w);
        CS::store_u(u_c, uint32_t(p), cn, hi, lo);
        CS::store_v(v_c, uint32_t(p), w);
        m_c[p] = m_grid[g] | P.cabs[p];
    } else {
        CS::load_u(u_c, uint32_t(p), cn, hi, lo);
        CS::load_v(v_c, uint32_t(p), w);
        S::store_u(u_grid, g, P.nsites, hi, lo);
        S::store_v(v_grid, g, P.nsites, w);
        m_grid[g] = m_c[p] & ~P.cabs[p];
    }
}

// Interior steps of a small 2D lattice in one launch: one workgroup keeps
// the whole state in LDS (two displacement buffers, velocities, flags and
// break bits, in the global layouts) and runs `nsteps` interior steps with
// a barrier between steps, then writes the state back (displacements to
// u_out).  Each step runs the gather kernel's per-site code on the LDS
// copy, so the results are bitwise those of nsteps gather launches; what
// it saves is a launch per step.
template <int PREC>
__global__ __launch_bounds__(kSmallBlock) void k_small_mid(StepParams P, int nsteps, int step_local) {
    using R = typename State<2, PREC>::R;
    using TTy = typename TT<PREC>::type;
    constexpr int VB = 2 * int(sizeof(R));  // velocity record
    extern __shared__ __attribute__((aligned(16))) char small_lds[];
    __shared__ TTy tt[kMaxTypes];
    __shared__ double mass_s[LSM_MAX_PHASES];
    __shared__ R imass_s[LSM_MAX_PHASES];
    const int ns = int(P.nsites);
    char *const uA = small_lds;
    char *const uB = uA + size_t(ns) * 16;
    char *const vv = uB + size_t(ns) * 16;
    uint8_t *const fl = reinterpret_cast<uint8_t *>(vv + size_t(ns) * VB);
    uint8_t *const mk = fl + ns;
    for (int t = threadIdx.x; t < kMaxTypes; t += blockDim.x) tt[t] = TT<PREC>::make(P.types[t]);
    if (threadIdx.x < LSM_MAX_PHASES) {
        mass_s[threadIdx.x] = P.mass[threadIdx.x];
        imass_s[threadIdx.x] = R(1.0 / P.mass[threadIdx.x]);
    }
    // both displacement buffers start as u_in (void sites are never
    // written, so either buffer can be the last)
    for (int g = threadIdx.x; g < ns; g += blockDim.x) {
        const uint4 u = reinterpret_cast<const uint4 *>(P.u_in)[g];
        reinterpret_cast<uint4 *>(uA)[g] = u;
        reinterpret_cast<uint4 *>(uB)[g] = u;
        if constexpr (VB == 16)
            reinterpret_cast<uint4 *>(vv)[g] = reinterpret_cast<const uint4 *>(P.v)[g];
        else
            reinterpret_cast<uint2 *>(vv)[g] = reinterpret_cast<const uint2 *>(P.v)[g];
        fl[g] = P.flags[g];
        mk[g] = reinterpret_cast<const uint8_t *>(P.mask)[g];
    }
    __syncthreads();
    StepParams L = P;
    L.flags = fl;
    L.mask = mk;
    L.v = vv;
    for (int s = 0; s < nsteps; ++s) {
        L.u_in = (s & 1) ? uB : uA;
        L.u_out = (s & 1) ? uA : uB;
        for (int g = threadIdx.x; g < ns; g += blockDim.x) {
            const uint8_t fp = fl[g];
            if (fp == kVoid) continue;
            double red[1] = {0.0};
            step_site<2, PREC, kMid, LSM_SPRING_LINEAR>(L, tt, mass_s, imass_s, g, g % P.nx, g / P.nx, 0, fp, red,
                                                        step_local + s);
        }
        __syncthreads();
    }
    const char *uf = (nsteps & 1) ? uB : uA;
    for (int g = threadIdx.x; g < ns; g += blockDim.x) {
        reinterpret_cast<uint4 *>(P.u_out)[g] = reinterpret_cast<const uint4 *>(uf)[g];
        if constexpr (VB == 16)
            reinterpret_cast<uint4 *>(P.v)[g] = reinterpret_cast<const uint4 *>(vv)[g];
        else
            reinterpret_cast<uint2 *>(P.v)[g] = reinterpret_cast<const uint2 *>(vv)[g];
        reinterpret_cast<uint8_t *>(P.mask)[g] = mk[g];
    }
}

// ------------------------------------------------------- increment kernel
template <int DIM, int PREC>
__global__ __launch_bounds__(256) void k_increment(StepParams P, double eps_new, double d_eps,
                                                   int inc, int affine) {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (g == 0) {
        P.ctl->eps = eps_new;
        P.ctl->inc = inc;
        P.ctl->step_base = 0;
        // a constant loading rate continues from the new strain
        P.ctl->rate_eps0 = eps_new;
        P.ctl->rate_s0 = 0;
    }
    if (g >= P.nsites) return;
    const uint8_t f = P.flags[g];
    if (f == kVoid) return;
    const int i = int(g % P.nx);
    const double c = double(i) * P.a;  // load coordinate of the site's column
    R hi[DIM], lo[DIM];
    S::load_u(P.u_in, int(g), P.nsites, hi, lo);
    if (flag_grip(f)) {
        const double ux = eps_new * c + 0.0;  // +0, not -0, on the origin column under compression
        hi[0] = R(ux);
        lo[0] = R(ux - double(hi[0]));
#pragma unroll
        for (int cc = 1; cc < DIM; ++cc) { hi[cc] = R(0); lo[cc] = R(0); }
        R z[DIM];
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) z[cc] = R(0);
        S::store_v(P.v, int(g), P.nsites, z);
        S::store_v(P.acc, int(g), P.nsites, z);
    } else if (affine) {
        if constexpr (PREC == 1) {
            const double ux = (double(hi[0]) + double(lo[0])) + d_eps * c;
            hi[0] = R(ux);
            lo[0] = R(ux - double(hi[0]));
        } else {
            hi[0] = hi[0] + d_eps * c;
        }
    }
    S::store_u(P.u_in, int(g), P.nsites, hi, lo);
}

// ---------------------------------------------- kick + drift (no forces)
// Continues a relaxation from a full step: v += dt/2 a, u += dt v.
template <int DIM, int PREC>
__global__ __launch_bounds__(256) void k_kick_drift(StepParams P) {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (g >= P.nsites) return;
    const uint8_t f = P.flags[g];
    if (f == kVoid || flag_grip(f)) return;
    const R h = R(0.5 * P.dt), dt = R(P.dt);
    R hi[DIM], lo[DIM], w[DIM], acc[DIM];
    S::load_u(P.u_in, int(g), P.nsites, hi, lo);
    S::load_v(P.v, int(g), P.nsites, w);
    S::load_v(P.acc, int(g), P.nsites, acc);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        w[c] = w[c] + h * acc[c];
        comp_add(hi[c], lo[c], dt * w[c]);
    }
    S::store_u(P.u_in, int(g), P.nsites, hi, lo);
    S::store_v(P.v, int(g), P.nsites, w);
}

// ------------------------------------------- constant-rate grip motion
// The paper's loading (Section 3.1: the boundary particles move apart along
// x at a constant strain rate; Section 2.3: the boundary displacement is the
// first operation of every time step).  Step S of the increment sees the
// grips at X0_x + eps_S i a with eps_S = eps0 + (S - S0) (rate dt), where
// eps0 was the strain at step S0 (the rate was set, or the increment
// began); the product and the sum are rounded separately, as written.  One
// thread per grip-column site (first and last column of every row).
template <int DIM, int PREC>
__global__ __launch_bounds__(256) void k_grips(StepParams P, int step_local) {
    using S = State<DIM, PREC>;
    using R = typename S::R;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int steps = P.ctl->step_base + step_local - P.ctl->rate_s0;
    const double eps = __dadd_rn(P.ctl->rate_eps0, __dmul_rn(double(steps), P.ctl->rate_de));
    if (t == 0) P.ctl->eps = eps;
    if (t >= 2 * int64_t(P.ny) * P.nz) return;
    const int i = (t & 1) ? P.nx - 1 : 0;
    const int64_t g = i + int64_t(P.nx) * (t >> 1);
    const uint8_t f = P.flags[g];
    if (f == kVoid || !flag_grip(f)) return;
    const double ux = eps * (double(i) * P.a) + 0.0;
    R hi[DIM], lo[DIM];
    hi[0] = R(ux);
    lo[0] = R(ux - double(hi[0]));
#pragma unroll
    for (int c = 1; c < DIM; ++c) { hi[c] = R(0); lo[c] = R(0); }
    S::store_u(P.u_in, int(g), P.nsites, hi, lo);
}

// ------------------------------------------------------- record finalize
__global__ __launch_bounds__(kBlock) void k_finalize(StepParams P, DevRecord *rec, double omega,
                                                     int nsteps, int dim) {
    __shared__ double lds[kNumPartials][kBlock / 64];
    double vals[kNumPartials];
#pragma unroll
    for (int v = 0; v < kNumPartials; ++v) vals[v] = 0.0;
    for (int b = threadIdx.x; b < P.red_blocks; b += kBlock) {
#pragma unroll
        for (int v = 0; v < kNumPartials; ++v) vals[v] += P.partials[int64_t(b) * kNumPartials + v];
    }
    block_sum(vals, lds);
    if (threadIdx.x == 0) {
        DevRecord r;
        r.eps = P.ctl->eps;
        bool finite = isfinite(vals[18]) && isfinite(vals[19]);
        for (int aa = 0; aa < 3; ++aa)
            for (int bb = 0; bb < 3; ++bb) {
                double s = 0.0;
                if (aa < dim && bb < dim) s = (vals[aa * 3 + bb] - vals[9 + aa * 3 + bb]) / omega;
                r.sigma[aa * 3 + bb] = s;
                finite = finite && isfinite(s);
            }
        r.pe = vals[18];
        r.ke = vals[19];
        const uint32_t ne = P.ctl->n_events;
        r.n_broken = int64_t(ne < P.ev_cap ? ne : P.ev_cap);
        r.increment = P.ctl->inc;
        r.step = P.ctl->step_base + nsteps;
        r.status = finite ? LSM_OK : LSM_EUNSTABLE;
        r.reserved = 0;
        *rec = r;
        P.ctl->step_base += nsteps;
    }
}


// ------------------------------------------------------- 2D row sweep
// Each wavefront owns kSweepCols columns of a vertical strip (plus one halo
// column on each side) and a chunk of rows, which it sweeps upward.  Per row
// a lane loads only its own site; the east neighbour and the sites of the
// row above come from adjacent lanes through DPP moves.  Every lane
// evaluates the three forward springs of its site (east, upper-left,
// upper-right) once; the three backward forces of a site are the negated
// forward forces of its west neighbour (this row, adjacent lane) and of its
// two lower neighbours (previous row, carried in registers).  The force sum
// has a fixed order per site, so results do not depend on the launch shape.

template <int T, int N, class F>
__device__ __attribute__((always_inline)) inline void unroll_rows(F &&f) {
    if constexpr (T < N) {
        f(std::integral_constant<int, T>{});
        unroll_rows<T + 1, N>(f);
    }
}

template <class R>
struct SweepRow {
    R uh[2], ul[2], v[2];
    int f, m;
};

template <int PREC, bool GRIP = false>
__device__ inline void load_sweep_row(const StepParams &P, const SweepItem &it, int i, bool col_ok, int jj,
                                      SweepRow<typename State<2, PREC>::R> &r, double geps = 0.0) {
    // Loads are unconditional from always-valid addresses, so no branch
    // joins on a pending load and no select waits for one.  Off the
    // specimen a lane reads its flag and break bits from the sentinel site
    // after the last one (void, no bits) and its displacement and velocity
    // from the specimen's first site: springs with a void end and unowned
    // sites never use them.  Offsets are 32-bit and relative to the
    // specimen's first site, whose address is uniform over the wavefront
    // (the sweeps run lattices and batches of fewer than 2^28 sites).
    using R = typename State<2, PREC>::R;
    const bool ok = col_ok && jj >= 0 && jj < it.ny;
    const uint32_t g = ok ? uint32_t(i + it.nx * jj) : 0u;
    const uint32_t gf = ok ? g : uint32_t(P.nsites - it.base);
    const char *ub = static_cast<const char *>(P.u_in) + size_t(it.base) * 16u + g * 16u;
    if constexpr (PREC == 1) {
        const float4 t = *reinterpret_cast<const float4 *>(ub);
        r.uh[0] = t.x; r.uh[1] = t.y; r.ul[0] = t.z; r.ul[1] = t.w;
    } else {
        const double2 t = *reinterpret_cast<const double2 *>(ub);
        r.uh[0] = t.x; r.uh[1] = t.y; r.ul[0] = 0.0; r.ul[1] = 0.0;
    }
    r.f = (P.flags + it.base)[gf];
    r.m = (reinterpret_cast<const uint8_t *>(P.mask) + it.base)[gf];
    if constexpr (GRIP) {
        if (r.f != kVoid && flag_grip(r.f) != 0) {
            // constant-rate loading: the grip's displacement at strain geps,
            // the value the grip kernel would have stored (the step carries it over)
            const double ux = geps * (double(i) * P.a) + 0.0;
            r.uh[0] = R(ux);
            r.ul[0] = R(ux - double(r.uh[0]));
            r.uh[1] = R(0);
            r.ul[1] = R(0);
        }
    }
    // the velocity too, also on the halo row below the chunk that is never
    // advanced: one more load there costs less than the branch around it
    const char *vb = static_cast<const char *>(P.v) + size_t(it.base) * (2 * sizeof(R)) + g * uint32_t(2 * sizeof(R));
    if constexpr (PREC == 1) {
        const float2 t = *reinterpret_cast<const float2 *>(vb);
        r.v[0] = t.x; r.v[1] = t.y;
    } else {
        const double2 t = *reinterpret_cast<const double2 *>(vb);
        r.v[0] = t.x; r.v[1] = t.y;
    }
}

// Work item of wavefront w: computed for a single lattice, read from the
// item table for a batch.  Returns false for wavefronts without work.
template <int BATCH>
__device__ inline bool sweep_item(const StepParams &P, int w, SweepItem &it) {
    if constexpr (BATCH) {
        if (w >= *P.n_items) return false;
        it = P.items[w];
    } else {
        if (w >= P.sw_nwork) return false;
        const int s = w % P.sw_strips;
        const int c = w / P.sw_strips;
        it.base = 0;
        it.nx = P.nx;
        it.ny = P.ny;
        it.i0 = s * kSweepCols - 1;
        it.j0 = c * P.sw_rows;
        it.j1 = min(it.j0 + P.sw_rows, P.ny);
        it.strip = s;
        it.strips = P.sw_strips;
        it.pbase = 0;
        it.spec = 0;
    }
    return true;
}

// One forward spring of site p towards q (lattice vector (ex, ey)).  Returns
// the force on p in f (zero if absent or broken), present = both ends are
// particles, brk = broken at this evaluation, margin = (r - rc) / rc when
// brk (left unset otherwise), ti = type index (meaningful when present).
// The FP32 form runs the same instructions on every lane and masks absent
// and broken springs at the end; only the FP64 test near rc branches.
template <int PREC, class TTy>
__device__ inline void fwd_spring(const TTy *tt, const TypeRec *types, int fp, int mask, int d,
                                  typename State<2, PREC>::R ex, typename State<2, PREC>::R ey,
                                  double ex64, double ey64, const typename State<2, PREC>::R *ph,
                                  const typename State<2, PREC>::R *pl,
                                  const typename State<2, PREC>::R *qh,
                                  const typename State<2, PREC>::R *ql, int fq, bool edge_ok,
                                  typename State<2, PREC>::R *f, int &present, int &brk,
                                  double &margin, int &ti) {
    using R = typename State<2, PREC>::R;
    present = (fp != kVoid) && (fq != kVoid);
    brk = 0;
    if constexpr (PREC == 1) {
        // phases are below LSM_MAX_PHASES = 8, so masking keeps void lanes in
        // the table
        ti = (fp & 7) * LSM_MAX_PHASES + (fq & 7);
        // the break bits also mark springs that do not exist (void or
        // off-lattice neighbour, void site), so one bit decides; a lane whose
        // neighbour lies across the wavefront edge is never owned and skips it
        const bool act = edge_ok && !(mask & (1 << d));
        R dv[2];
        dv[0] = ex + ((qh[0] - ph[0]) + (ql[0] - pl[0]));
        dv[1] = (qh[1] - ph[1]) + (ql[1] - pl[1]);
        if (d != 0) dv[1] = ey + dv[1];  // the east spring has ey = 0
        const R r2 = dv[0] * dv[0] + dv[1] * dv[1];
        const TTy T = tt[ti];
        if (act && r2 > T.z) {
            const double dx = ex64 + ((double(qh[0]) - double(ph[0])) + (double(ql[0]) - double(pl[0])));
            const double dy = ey64 + ((double(qh[1]) - double(ph[1])) + (double(ql[1]) - double(pl[1])));
            const double r64 = sqrt(dx * dx + dy * dy);
            const double rc = types[ti].rc64;
            brk = r64 > rc;
            margin = (r64 - rc) / rc;
        }
        // r2 is a normal number on every active spring; other lanes are
        // masked below whatever rsq returns for them
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float coef = fmaf(-T.y, rinv, T.x);  // k (r - r0) / r
        const bool ok = act && !brk;
        f[0] = ok ? coef * dv[0] : R(0);
        f[1] = ok ? coef * dv[1] : R(0);
    } else {
        f[0] = R(0);
        f[1] = R(0);
        ti = present ? flag_phase(fp) * LSM_MAX_PHASES + flag_phase(fq) : 0;
        if (!present || (mask & (1 << d))) return;
        R dv[2];
        dv[0] = ex + ((qh[0] - ph[0]) + (ql[0] - pl[0]));
        dv[1] = ey + ((qh[1] - ph[1]) + (ql[1] - pl[1]));
        const R r2 = dv[0] * dv[0] + dv[1] * dv[1];
        const TTy T = tt[ti];
        const double r = sqrt(r2);
        brk = r > T.z;
        if (brk) {
            margin = (r - T.z) / T.z;
            return;
        }
        const double coef = T.x * (r - T.y) / r;
        f[0] = coef * dv[0];
        f[1] = coef * dv[1];
    }
}

// FP64 virial and potential energy of one intact spring (Eq. 7, Eq. 1).
template <class R>
__device__ inline void spring_stress64(const TypeRec &T, double ex64, double ey64, const R *ph,
                                       const R *pl, const R *qh, const R *ql, double *red) {
    double d[2];
    d[0] = ex64 + ((double(qh[0]) - double(ph[0])) + (double(ql[0]) - double(pl[0])));
    d[1] = ey64 + ((double(qh[1]) - double(ph[1])) + (double(ql[1]) - double(pl[1])));
    const double r = sqrt(d[0] * d[0] + d[1] * d[1]);
    const double coef = T.k64 * (r - T.r0_64) / r;
#pragma unroll
    for (int aa = 0; aa < 2; ++aa)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) red[aa * 3 + bb] += d[aa] * (coef * d[bb]);
    red[18] += 0.5 * T.k64 * (r - T.r0_64) * (r - T.r0_64);
}

// The three forward springs of a swept row (east, upper-left, upper-right),
// evaluated per lane from the row (rc) and the row above (ru); neighbour
// sites come from adjacent lanes through DPP moves, so every lane of the
// wavefront must call this.
template <class R>
struct RowSprings {
    R eh[2], el[2], ulh[2], ull[2], urh[2], url[2];  // neighbour displacements (stress)
    R fe[2], ful[2], fur[2];                         // forces on this site
    int pe, pul, pur, be, bul, bur, te, tul, tur;    // present, broken now, type index
    double me, mul, mur;                             // break margins
    int nb;                                          // bits 0..2: broken at this evaluation
    int fb;                                          // bits 0..2: broken now or before
};

template <int PREC, int PAR, class TTy>
__device__ inline void row_springs(const TTy *tt, const TypeRec *types,
                                   const SweepRow<typename State<2, PREC>::R> &rc,
                                   const SweepRow<typename State<2, PREC>::R> &ru,
                                   RowSprings<typename State<2, PREC>::R> &o, double a64, bool not_last,
                                   bool not_first) {
    using R = typename State<2, PREC>::R;
    const R a = R(a64), hy = R(kHalfSqrt3 * a64);
    const double hy64 = kHalfSqrt3 * a64;
    const R half_a = R(0.5) * a;
    int ef, ulf, urf;
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        o.eh[cc] = lane_next(rc.uh[cc]);
        o.el[cc] = PREC ? lane_next(rc.ul[cc]) : R(0);
    }
    ef = lane_next(rc.f);
    if constexpr (PAR == 0) {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            o.ulh[cc] = lane_prev(ru.uh[cc]);
            o.ull[cc] = PREC ? lane_prev(ru.ul[cc]) : R(0);
            o.urh[cc] = ru.uh[cc];
            o.url[cc] = ru.ul[cc];
        }
        ulf = lane_prev(ru.f);
        urf = ru.f;
    } else {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            o.ulh[cc] = ru.uh[cc];
            o.ull[cc] = ru.ul[cc];
            o.urh[cc] = lane_next(ru.uh[cc]);
            o.url[cc] = PREC ? lane_next(ru.ul[cc]) : R(0);
        }
        ulf = ru.f;
        urf = lane_next(ru.f);
    }
    fwd_spring<PREC>(tt, types, rc.f, rc.m, 0, a, R(0), a64, 0.0, rc.uh, rc.ul, o.eh, o.el, ef, not_last, o.fe, o.pe,
                     o.be, o.me, o.te);
    fwd_spring<PREC>(tt, types, rc.f, rc.m, 1, -half_a, hy, -0.5 * a64, hy64, rc.uh, rc.ul, o.ulh, o.ull, ulf,
                     PAR == 0 ? not_first : true,
                     o.ful, o.pul, o.bul, o.mul, o.tul);
    fwd_spring<PREC>(tt, types, rc.f, rc.m, 2, half_a, hy, 0.5 * a64, hy64, rc.uh, rc.ul, o.urh, o.url, urf,
                     PAR == 0 ? true : not_last,
                     o.fur, o.pur, o.bur, o.mur, o.tur);
    o.nb = o.be | (o.bul << 1) | (o.bur << 2);
    o.fb = o.nb | (rc.m & 7);
}

// Total force on the lane's site: its forward springs, minus the forward
// forces of its west neighbour (adjacent lane) and of its two lower
// neighbours (carried from the row below: pUL, pUR, and pbrk = their
// upper-left / upper-right "broken now or before" bits), in a fixed order;
// and its break mask after this evaluation.  The backward bits come from
// the neighbours' broken-now-or-before bits, so they do not depend on
// whether the owner of a neighbouring site has already stored its new bits
// when this lane reads them.  DPP moves: every lane must call this.
template <int PAR, class R>
__device__ inline void row_force(const RowSprings<R> &o, const R *pUL, const R *pUR, int pbrk, int m,
                                 R *F, int &newmask) {
    R gW[2], gDR[2], gDL[2];
    int bW, bDR, bDL;
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) gW[cc] = lane_prev(o.fe[cc]);
    bW = lane_prev(o.fb) & 1;
    if constexpr (PAR == 0) {
        // lower-right neighbour is this lane, lower-left the previous lane
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            gDR[cc] = pUL[cc];
            gDL[cc] = lane_prev(pUR[cc]);
        }
        bDR = pbrk & 1;
        bDL = (lane_prev(pbrk) >> 1) & 1;
    } else {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            gDR[cc] = lane_next(pUL[cc]);
            gDL[cc] = pUR[cc];
        }
        bDR = lane_next(pbrk) & 1;
        bDL = (pbrk >> 1) & 1;
    }
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) F[cc] = ((((o.fe[cc] + o.ful[cc]) + o.fur[cc]) - gW[cc]) - gDR[cc]) - gDL[cc];
    newmask = m | o.nb | (bW << 3) | (bDR << 4) | (bDL << 5);
}

// GRIP: constant-rate loading, where each row load places the grips at this
// step's strain (interior steps only; compiled out of every other sweep)
template <int PREC, int MODE, int PF, int BATCH, bool GRIP>
__device__ __attribute__((always_inline)) inline void sweep2d_body(const StepParams &P, int step_local) {
    using S = State<2, PREC>;
    using R = typename S::R;
    using TTy = typename TT<PREC>::type;
    __shared__ TTy tt[kMaxTypes];
    __shared__ double mass_s[LSM_MAX_PHASES];
    __shared__ R imass_s[LSM_MAX_PHASES];  // R(1 / m), once per workgroup
    __shared__ double red_lds[MODE == kEnd ? kNumPartials : 1][kBlock / 64];
    for (int t = threadIdx.x; t < kMaxTypes; t += kBlock) tt[t] = TT<PREC>::make(P.types[t]);
    if (threadIdx.x < LSM_MAX_PHASES) {
        mass_s[threadIdx.x] = P.mass[threadIdx.x];
        imass_s[threadIdx.x] = R(1.0 / P.mass[threadIdx.x]);
    }
    __syncthreads();

    double red[MODE == kEnd ? kNumPartials : 1];
#pragma unroll
    for (int v = 0; v < (MODE == kEnd ? kNumPartials : 1); ++v) red[v] = 0.0;

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int per = P.sw_nblocks >> 3;
    const int L = int(blockIdx.x & 7) * per + int(blockIdx.x >> 3);
    const int w = L * (kBlock / 64) + wv;
    SweepItem it;
    if (sweep_item<BATCH>(P, w, it)) {
        const int i = it.i0 + lane;
        const bool col_ok = i >= 0 && i < it.nx;
        const bool own_lane = col_ok && lane >= 1 && lane <= kSweepCols;
        const bool not_last = lane != 63, not_first = lane != 0;  // DPP neighbours inside the wavefront
        const int j0 = it.j0;
        const int j1 = it.j1;
        const int jstart = j0 > 0 ? j0 - 1 : 0;
        const int js = jstart & ~1;  // even: the parity of each unrolled row is a constant
        const double a64 = P.a, hy64 = kHalfSqrt3 * P.a;
        // strain of this step under constant-rate loading (the grip kernel's formula)
        double geps = 0.0;
        if constexpr (GRIP) {
            const int steps = P.ctl->step_base + step_local - P.ctl->rate_s0;
            geps = __dadd_rn(P.ctl->rate_eps0, __dmul_rn(double(steps), P.ctl->rate_de));
        }

        R pUL[2] = {R(0), R(0)}, pUR[2] = {R(0), R(0)};
        int pbrk = 0;
        // Row j is computed from rc (row j) and ru (row j + 1) while rn
        // receives row j + 2; the three buffers rotate roles so that no
        // register copy forces an early wait on the prefetched row.
        auto row_step = [&](auto parc, int j, SweepRow<R> &rc, SweepRow<R> &ru,
                            SweepRow<R> &rn) __attribute__((always_inline)) {
            constexpr int PAR = decltype(parc)::value;
            load_sweep_row<PREC, GRIP>(P, it, i, col_ok, j + PF + 1 <= j1 ? j + PF + 1 : -1, rn, geps);
            RowSprings<R> o;
            row_springs<PREC, PAR>(tt, P.types, rc, ru, o, P.a, not_last, not_first);
            const R *eh = o.eh, *el = o.el, *ulh = o.ulh, *ull = o.ull, *urh = o.urh, *url = o.url;
            const R *fe = o.fe, *ful = o.ful, *fur = o.fur;
            const int pe = o.pe, pul = o.pul, pur = o.pur, be = o.be, bul = o.bul, bur = o.bur;
            const int te = o.te, tul = o.tul, tur = o.tur;
            const double me = o.me, mul = o.mul, mur = o.mur;
            const int nb = o.nb;
            if (j >= j0) {
                R F[2];
                int newmask;
                row_force<PAR>(o, pUL, pUR, pbrk, rc.m, F, newmask);
                if (own_lane && rc.f != kVoid) {
                    const uint32_t g = uint32_t(it.base + i + it.nx * j);
                    if (newmask != rc.m) {
                        reinterpret_cast<uint8_t *>(P.mask)[g] = uint8_t(newmask);
                        if constexpr (BATCH) {
                            // batches keep a per-specimen count instead of a log
                            const int nnew = be + bul + bur;
                            if (nnew) atomicAdd(&P.spec_broken[it.spec], uint32_t(nnew));
                        } else {
                        const int brks[3] = {be, bul, bur};
                        const double mgs[3] = {me, mul, mur};
                        const int pres[3] = {pe, pul, pur};
                        int rank = 0;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            if (brks[d]) {
                                const uint32_t idx = event_slot(P.ctl);
                                if (idx < P.ev_cap) {
                                    lsm_event ev;
                                    ev.increment = P.ctl->inc;
                                    ev.step = P.ctl->step_base + step_local;
                                    ev.spring_id = int64_t(P.sbase[g]) + rank;
                                    ev.margin = mgs[d];
                                    P.events[idx] = ev;
                                }
                            }
                            rank += pres[d];
                        }
                        }
                    }
                    if constexpr (MODE == kEnd) {
                        const int mk = newmask;
                        if (pe && !(mk & 1)) spring_stress64(P.types[te], a64, 0.0, rc.uh, rc.ul, eh, el, red);
                        if (pul && !(mk & 2))
                            spring_stress64(P.types[tul], -0.5 * a64, hy64, rc.uh, rc.ul, ulh, ull, red);
                        if (pur && !(mk & 4))
                            spring_stress64(P.types[tur], 0.5 * a64, hy64, rc.uh, rc.ul, urh, url, red);
                    }
                    integrate_site<2, PREC, MODE>(P, RowStore<PREC>{g}, uint8_t(rc.f),
                                                  mass_s[flag_phase(rc.f)],
                                                  imass_s[flag_phase(rc.f)], rc.uh,
                                                  rc.ul, F, rc.v, red);
                }
                if constexpr (MODE == kEnd) {
                    // one partial per (row, strip): the reduction order does not
                    // depend on how rows are chunked over wavefronts
#pragma unroll
                    for (int v = 0; v < kNumPartials; ++v) {
                        const double t = wave_sum(red[v]);
                        if (lane == 0)
                            P.partials[(int64_t(it.pbase) + int64_t(j) * it.strips + it.strip) * kNumPartials + v] = t;
                        red[v] = 0.0;
                    }
                }
            }
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                pUL[cc] = ful[cc];
                pUR[cc] = fur[cc];
            }
            pbrk = (o.fb >> 1) & 3;
        };

        // K (even) rotating row buffers: row j lives in B[(j - js) % K]; the
        // step for row j prefetches row j + PF + 1.  A row below jstart
        // (js = jstart - 1) is loaded as void: it has no springs and no work.
        constexpr int K = (PF + 3) & ~1;
        SweepRow<R> B[K];
#pragma unroll
        for (int t = 0; t <= PF; ++t) {
            const int jj = js + t;
            load_sweep_row<PREC, GRIP>(P, it, i, col_ok, jj >= jstart && jj <= j1 ? jj : -1, B[t], geps);
        }
        for (int j = js; j < j1; j += K) {
            unroll_rows<0, K>([&](auto tc) __attribute__((always_inline)) {
                constexpr int t = decltype(tc)::value;
                if (j + t < j1)
                    row_step(std::integral_constant<int, t & 1>{}, j + t, B[t], B[(t + 1) % K],
                             B[(t + PF + 1) % K]);
            });
        }
    }
    (void)red_lds;
}

template <int PREC, int MODE, int PF, int BATCH>
__global__ __launch_bounds__(kBlock) void k_sweep2d(StepParams P, int step_local) {
    sweep2d_body<PREC, MODE, PF, BATCH, false>(P, step_local);
}

// interior step under constant-rate loading (single lattices)
template <int PREC, int PF>
__global__ __launch_bounds__(kBlock) void k_sweep2d_rate(StepParams P, int step_local) {
    sweep2d_body<PREC, kMid, PF, 0, true>(P, step_local);
}

// Two interior time steps per launch: temporal blocking of the row sweep.
// Stage A advances the rows read from memory by one step and keeps each
// row's new state (displacement, velocity, break bits) in registers; stage
// B, one row behind, advances that state by a second step and writes it.
// Stage A is valid on lanes 1..62 and stage B on lanes 2..61, so a wavefront
// owns 60 columns (kSweepCols2) and rows j0..j1-1; stage A also advances
// rows j0-1 and j1 and evaluates the forward springs of row j0-2, whose
// forces act on row j0-1.  Velocities and break bits are read from P.v /
// P.mask and written to P.v_out / P.mask_out: neighbouring wavefronts read
// the sites a wavefront owns (as their halo rows and columns) during the
// same launch, so nothing they read may be updated in place.  Every site
// goes through exactly the operations of two single-step launches (shared
// helpers, same order), so the state is bitwise the same; memory is read
// and written once per two steps.  FP32-compensated lattices only.
template <int PREC>
__device__ inline void log_breaks(const StepParams &P, int g, const RowSprings<typename State<2, PREC>::R> &o,
                                  int step) {
    const int brks[3] = {o.be, o.bul, o.bur};
    const double mgs[3] = {o.me, o.mul, o.mur};
    const int pres[3] = {o.pe, o.pul, o.pur};
    int rank = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (brks[d]) {
            const uint32_t idx = event_slot(P.ctl);
            if (idx < P.ev_cap) {
                lsm_event ev;
                ev.increment = P.ctl->inc;
                ev.step = P.ctl->step_base + step;
                ev.spring_id = int64_t(P.sbase[g]) + rank;
                ev.margin = mgs[d];
                P.events[idx] = ev;
            }
        }
        rank += pres[d];
    }
}

template <int PREC, int PF, int BATCH>
__device__ __attribute__((always_inline)) inline void sweep2d_x2_body(const StepParams &P, int step_local) {
    using S = State<2, PREC>;
    using R = typename S::R;
    using TTy = typename TT<PREC>::type;
    __shared__ TTy tt[kMaxTypes];
    // 1 / m by the low six flag bits (phase, grip), zero for grips and void
    // sites: every lane runs the update, which then leaves a grip's state
    // exactly as it was (zero velocity, zero drift into a normalised
    // compensated pair)
    __shared__ R imass_f[64];
    for (int t = threadIdx.x; t < kMaxTypes; t += kBlock) tt[t] = TT<PREC>::make(P.types[t]);
    if (threadIdx.x < 64) {
        const int ph = threadIdx.x & 15, grip = (threadIdx.x >> 4) & 3;
        imass_f[threadIdx.x] = (grip == 0 && ph < LSM_MAX_PHASES) ? R(1.0 / P.mass[ph]) : R(0);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int per = P.sw2_nblocks >> 3;
    const int Lb = int(blockIdx.x & 7) * per + int(blockIdx.x >> 3);
    const int w = Lb * (kBlock / 64) + wv;
    SweepItem it;
    if constexpr (BATCH) {
        if (w >= *P.n_items2) return;  // whole wavefronts; no barrier follows
        it = P.items2[w];
    } else {
        if (w >= P.sw2_nwork) return;
        it.base = 0;
        it.nx = P.nx;
        it.ny = P.ny;
        it.i0 = (w % P.sw2_strips) * kSweepCols2 - 2;
        it.j0 = (w / P.sw2_strips) * P.sw_rows;
        it.j1 = min(it.j0 + P.sw_rows, P.ny);
    }
    const int i = it.i0 + lane;
    const bool col_ok = i >= 0 && i < it.nx;
    const bool own = col_ok && lane >= 2 && lane <= kSweepCols2 + 1;
    const bool not_last = lane != 63, not_first = lane != 0;  // DPP neighbours inside the wavefront
    const int j0 = it.j0, j1 = it.j1;
    const int ja = j0 >= 2 ? j0 - 2 : 0;
    const int a0 = ja & ~1;  // even: the parity of each unrolled row is a constant
    const R h = R(0.5 * P.dt), dt = R(P.dt), gam = R(P.gamma);

    R aUL[2] = {R(0), R(0)}, aUR[2] = {R(0), R(0)};  // stage A: forces carried from the row below
    R bUL[2] = {R(0), R(0)}, bUR[2] = {R(0), R(0)};  // stage B
    int abrk = 0, bbrk = 0;

    // Row a: stage A at step s on rc (row a, advanced in place, so rc then
    // holds the stage-A state), ru = row a + 1, rn receives row a + PF + 1;
    // stage B at step s + 1 on row a - 1 from Aprev (its stage-A state).
    auto row_step = [&](auto parc, int a, SweepRow<R> &rc, const SweepRow<R> &ru, SweepRow<R> &rn,
                        const SweepRow<R> &Aprev) __attribute__((always_inline)) {
        constexpr int PAR = decltype(parc)::value;  // a & 1
        const int jn = a + PF + 1;
        load_sweep_row<PREC>(P, it, i, col_ok, jn <= j1 + 1 ? jn : -1, rn);
        // ---- stage A: row a, step s
        RowSprings<R> oa;
        row_springs<PREC, PAR>(tt, P.types, rc, ru, oa, P.a, not_last, not_first);
        SweepRow<R> &Acur = rc;
        if (a >= j0 - 1) {
            R F[2];
            int nm;
            row_force<PAR>(oa, aUL, aUR, abrk, rc.m, F, nm);
            Acur.m = nm;
            R acc[2];
            site_acc<2, PREC>(F, Acur.v, 0.0, imass_f[Acur.f & 63], gam, acc);
            mid_kick_drift<2, PREC>(Acur.uh, Acur.ul, Acur.v, acc, h, dt);
            if (own && a >= j0 && a < j1 && Acur.f != kVoid && oa.nb) {
                if constexpr (BATCH)  // batches keep a per-specimen count instead of a log
                    atomicAdd(&P.spec_broken[it.spec], uint32_t(oa.be + oa.bul + oa.bur));
                else
                    log_breaks<PREC>(P, i + it.nx * a, oa, step_local);
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            aUL[c] = oa.ful[c];
            aUR[c] = oa.fur[c];
        }
        abrk = (oa.fb >> 1) & 3;
        // ---- stage B: row a - 1, step s + 1, from the stage-A states
        const int b = a - 1;
        if (b >= j0 - 1) {
            RowSprings<R> ob;
            row_springs<PREC, PAR ^ 1>(tt, P.types, Aprev, Acur, ob, P.a, not_last, not_first);
            if (b >= j0) {
                R F[2];
                int nm;
                row_force<PAR ^ 1>(ob, bUL, bUR, bbrk, Aprev.m, F, nm);
                if (own && Aprev.f != kVoid) {
                    // offset from the specimen's first site (uniform base addresses)
                    const uint32_t g = uint32_t(i + it.nx * b);
                    (reinterpret_cast<uint8_t *>(P.mask_out) + it.base)[g] = uint8_t(nm);
                    if (ob.nb) {
                        if constexpr (BATCH)
                            atomicAdd(&P.spec_broken[it.spec], uint32_t(ob.be + ob.bul + ob.bur));
                        else
                            log_breaks<PREC>(P, g, ob, step_local + 1);  // one lattice: base 0
                    }
                    R uh[2], ul[2], v[2];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        uh[c] = Aprev.uh[c];
                        ul[c] = Aprev.ul[c];
                        v[c] = Aprev.v[c];
                    }
                    R acc[2];
                    site_acc<2, PREC>(F, v, 0.0, imass_f[Aprev.f & 63], gam, acc);
                    mid_kick_drift<2, PREC>(uh, ul, v, acc, h, dt);
                    const RowStore<PREC> st{g};
                    st.v(static_cast<char *>(P.v_out) + size_t(it.base) * (2 * sizeof(R)), v);
                    st.u(static_cast<char *>(P.u_out) + size_t(it.base) * 16u, uh, ul);
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                bUL[c] = ob.ful[c];
                bUR[c] = ob.fur[c];
            }
            bbrk = (ob.fb >> 1) & 3;
        }
    };

    // K (even) rotating row buffers: row a lives in B[(a - a0) % K]; the
    // step for row a prefetches row a + PF + 1 into B[(a - a0 + PF + 1) % K],
    // which with K >= PF + 3 is neither row a - 1 (stage B still reads it)
    // nor row a + 1.  A row below ja (a0 = ja - 1) is loaded as void: no
    // springs, and stage B skips the row below it.  B[K - 1] starts as a
    // void row: the stage-A state of row a0 - 1 seen by the first stage B.
    constexpr int K = (PF + 4) & ~1;
    SweepRow<R> B[K];
#pragma unroll
    for (int t = 0; t <= PF; ++t) {
        const int jj = a0 + t;
        load_sweep_row<PREC>(P, it, i, col_ok, jj >= ja && jj <= j1 + 1 ? jj : -1, B[t]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) B[K - 1].uh[c] = B[K - 1].ul[c] = B[K - 1].v[c] = R(0);
    B[K - 1].f = kVoid;
    B[K - 1].m = 0;
    for (int a = a0; a <= j1; a += K) {
        unroll_rows<0, K>([&](auto tc) __attribute__((always_inline)) {
            constexpr int t = decltype(tc)::value;
            if (a + t <= j1)
                row_step(std::integral_constant<int, t & 1>{}, a + t, B[t], B[(t + 1) % K], B[(t + PF + 1) % K],
                         B[(t + K - 1) % K]);
        });
    }
}

template <int PREC, int PF>
__global__ __launch_bounds__(kBlock) void k_sweep2d_x2(StepParams P, int step_local) {
    sweep2d_x2_body<PREC, PF, 0>(P, step_local);
}

// Batches.  With prefetch depth 1 the registers of the item-table variant
// fit five wavefronts per SIMD without spills (measured 3 % faster on the
// C4 batch); the single-lattice kernel and depth 2 would spill there.
template <int PREC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_sweep2d_x2_batch1(StepParams P,
                                                                                                      int step_local) {
    sweep2d_x2_body<PREC, 1, 1>(P, step_local);
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_sweep2d_x2_batch2(StepParams P, int step_local) {
    sweep2d_x2_body<PREC, 2, 1>(P, step_local);
}

template <int DIM, int PREC>
hipError_t launch_step_t(const StepParams &p, int mode, hipStream_t s, int step_local) {
    const dim3 grid(p.plist ? p.c_blocks : p.nblocks), block(kBlock);
    switch (mode) {
        case kStart: hipLaunchKernelGGL((k_step<DIM, PREC, kStart>), grid, block, 0, s, p, step_local); break;
        case kMid: hipLaunchKernelGGL((k_step<DIM, PREC, kMid>), grid, block, 0, s, p, step_local); break;
        case kEnd: hipLaunchKernelGGL((k_step<DIM, PREC, kEnd>), grid, block, 0, s, p, step_local); break;
        default: hipLaunchKernelGGL((k_step<DIM, PREC, kEval>), grid, block, 0, s, p, step_local); break;
    }
    return hipGetLastError();
}

template <int PREC, int PF, int BATCH>
hipError_t launch_sweep_pf(const StepParams &p, int mode, hipStream_t s, int step_local, int nblocks) {
    const dim3 grid(nblocks), block(kBlock);
    switch (mode) {
        case kStart: hipLaunchKernelGGL((k_sweep2d<PREC, kStart, PF, BATCH>), grid, block, 0, s, p, step_local); break;
        case kMid:
            if constexpr (BATCH == 0) {
                if (p.grip_rate) {
                    hipLaunchKernelGGL((k_sweep2d_rate<PREC, PF>), grid, block, 0, s, p, step_local);
                    break;
                }
            }
            hipLaunchKernelGGL((k_sweep2d<PREC, kMid, PF, BATCH>), grid, block, 0, s, p, step_local);
            break;
        default: hipLaunchKernelGGL((k_sweep2d<PREC, kEnd, PF, BATCH>), grid, block, 0, s, p, step_local); break;
    }
    return hipGetLastError();
}

template <int PREC, int BATCH>
hipError_t launch_sweep_t(const StepParams &p, int mode, hipStream_t s, int step_local, int nblocks) {
    // the prefetch depth only matters for the interior steps
    if (mode != kMid || p.sw_pf <= 1) return launch_sweep_pf<PREC, 1, BATCH>(p, mode, s, step_local, nblocks);
    if (p.sw_pf == 2) return launch_sweep_pf<PREC, 2, BATCH>(p, mode, s, step_local, nblocks);
    return launch_sweep_pf<PREC, 3, BATCH>(p, mode, s, step_local, nblocks);
}

// Increment for a batch: grips to eps * i * a, affine predictor elsewhere,
// over the owned sites of each active work item.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_increment_batch(StepParams P, double eps_new, double d_eps,
                                                            int inc, int affine) {
    using S = State<2, PREC>;
    using R = typename S::R;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.ctl->eps = eps_new;
        P.ctl->inc = inc;
        P.ctl->step_base = 0;
    }
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int w = int(blockIdx.x) * (kBlock / 64) + wv;
    SweepItem it;
    if (!sweep_item<1>(P, w, it)) return;
    const int i = it.i0 + lane;
    if (!(i >= 0 && i < it.nx && lane >= 1 && lane <= kSweepCols)) return;
    const double c = double(i) * P.a;
    for (int j = it.j0; j < it.j1; ++j) {
        const int g = it.base + i + it.nx * j;
        const uint8_t f = P.flags[g];
        if (f == kVoid) continue;
        R hi[2], lo[2];
        S::load_u(P.u_in, g, P.nsites, hi, lo);
        if (flag_grip(f)) {
            const double ux = eps_new * c + 0.0;  // +0, not -0, on the origin column under compression
            hi[0] = R(ux);
            lo[0] = R(ux - double(hi[0]));
            hi[1] = R(0);
            lo[1] = R(0);
            const R z[2] = {R(0), R(0)};
            S::store_v(P.v, g, P.nsites, z);
            S::store_v(P.acc, g, P.nsites, z);
        } else if (affine) {
            if constexpr (PREC == 1) {
                const double ux = (double(hi[0]) + double(lo[0])) + d_eps * c;
                hi[0] = R(ux);
                lo[0] = R(ux - double(hi[0]));
            } else {
                hi[0] = hi[0] + d_eps * c;
            }
        }
        S::store_u(P.u_in, g, P.nsites, hi, lo);
    }
}

// Per-specimen record: one workgroup per specimen sums its partials in a
// fixed order.
__global__ __launch_bounds__(kBlock) void k_finalize_batch(StepParams P, DevRecord *recs,
                                                           const SpecDesc *specs, int nsteps, int dim) {
    __shared__ double lds[kNumPartials][kBlock / 64];
    const SpecDesc sd = specs[blockIdx.x];
    double vals[kNumPartials];
#pragma unroll
    for (int v = 0; v < kNumPartials; ++v) vals[v] = 0.0;
    for (int b = threadIdx.x; b < sd.npart; b += kBlock) {
#pragma unroll
        for (int v = 0; v < kNumPartials; ++v)
            vals[v] += P.partials[(int64_t(sd.pbase) + b) * kNumPartials + v];
    }
    block_sum(vals, lds);
    if (threadIdx.x == 0) {
        DevRecord r;
        r.eps = P.ctl->eps;
        bool finite = isfinite(vals[18]) && isfinite(vals[19]);
        for (int aa = 0; aa < 3; ++aa)
            for (int bb = 0; bb < 3; ++bb) {
                double s = 0.0;
                if (aa < dim && bb < dim) s = (vals[aa * 3 + bb] - vals[9 + aa * 3 + bb]) / sd.omega;
                r.sigma[aa * 3 + bb] = s;
                finite = finite && isfinite(s);
            }
        r.pe = vals[18];
        r.ke = vals[19];
        r.n_broken = int64_t(P.spec_broken[blockIdx.x]);
        r.increment = P.ctl->inc;
        r.step = nsteps;
        r.status = finite ? LSM_OK : LSM_EUNSTABLE;
        r.reserved = 0;
        recs[blockIdx.x] = r;
    }
}

}  // namespace

hipError_t launch_sweep2d(const StepParams &p, int prec, int mode, hipStream_t s, int step_local) {
    return prec ? launch_sweep_t<1, 0>(p, mode, s, step_local, p.sw_nblocks)
                : launch_sweep_t<0, 0>(p, mode, s, step_local, p.sw_nblocks);
}

static int batch_blocks(int capacity) {
    const int wgs = (capacity + kBlock / 64 - 1) / (kBlock / 64);
    return ((wgs + 7) / 8) * 8;
}

hipError_t launch_sweep2d_batch(const StepParams &p, int prec, int mode, hipStream_t s, int step_local,
                                int capacity) {
    StepParams q = p;
    q.sw_nblocks = batch_blocks(capacity);
    return prec ? launch_sweep_t<1, 1>(q, mode, s, step_local, q.sw_nblocks)
                : launch_sweep_t<0, 1>(q, mode, s, step_local, q.sw_nblocks);
}

hipError_t launch_sweep2d_x2_batch(const StepParams &p, int prec, hipStream_t s, int step_local, int capacity2) {
    if (!prec) return hipErrorInvalidValue;  // FP32-compensated batches only
    StepParams q = p;
    q.sw2_nblocks = batch_blocks(capacity2);
    const dim3 grid(q.sw2_nblocks), block(kBlock);
    if (q.sw_pf >= 2) hipLaunchKernelGGL(k_sweep2d_x2_batch2<1>, grid, block, 0, s, q, step_local);
    else hipLaunchKernelGGL(k_sweep2d_x2_batch1<1>, grid, block, 0, s, q, step_local);
    return hipGetLastError();
}

hipError_t launch_increment_batch(const StepParams &p, int prec, hipStream_t s, double eps_new,
                                  double d_eps, int inc, int affine, int capacity) {
    const dim3 grid(unsigned((capacity + kBlock / 64 - 1) / (kBlock / 64))), block(kBlock);
    if (prec) hipLaunchKernelGGL((k_increment_batch<1>), grid, block, 0, s, p, eps_new, d_eps, inc, affine);
    else hipLaunchKernelGGL((k_increment_batch<0>), grid, block, 0, s, p, eps_new, d_eps, inc, affine);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const StepParams &p, int dim, hipStream_t s, DevRecord *recs,
                                 const SpecDesc *specs, int nspec, int nsteps) {
    if (nspec <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_batch, dim3(nspec), dim3(kBlock), 0, s, p, recs, specs, nsteps, dim);
    return hipGetLastError();
}

int sweep_waves_per_cu(int two_step, int prec, int pf) {
    // resident workgroups of the interior-step kernel per CU, in wavefronts
    int blocks = 0;
    hipError_t e;
    if (two_step)
        e = pf >= 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep2d_x2<1, 2>, kBlock, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep2d_x2<1, 1>, kBlock, 0);
    else if (prec)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep2d<1, kMid, 1, 0>, kBlock, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep2d<0, kMid, 1, 0>, kBlock, 0);
    return e == hipSuccess ? blocks * (kBlock / 64) : 0;
}

hipError_t launch_sweep2d_x2(const StepParams &p, int prec, hipStream_t s, int step_local) {
    const dim3 grid(p.sw2_nblocks), block(kBlock);
    if (!prec) return hipErrorInvalidValue;  // FP32-compensated lattices only
    if (p.sw_pf >= 2) hipLaunchKernelGGL((k_sweep2d_x2<1, 2>), grid, block, 0, s, p, step_local);
    else hipLaunchKernelGGL((k_sweep2d_x2<1, 1>), grid, block, 0, s, p, step_local);
    return hipGetLastError();
}

size_t small_lds_bytes(int64_t nsites, int prec) {
    return size_t(nsites) * size_t(32 + (prec ? 8 : 16) + 2);
}

hipError_t launch_small_mid(const StepParams &p, int prec, hipStream_t s, int nsteps, int step_local) {
    const size_t lds = small_lds_bytes(p.nsites, prec);
    if (p.nsites <= 0 || lds > kSmallLdsBytes || nsteps < 1) return hipErrorInvalidValue;
    const int threads = int(std::min<int64_t>(kSmallBlock, (p.nsites + 63) / 64 * 64));
    if (prec) hipLaunchKernelGGL((k_small_mid<1>), dim3(1), dim3(threads), lds, s, p, nsteps, step_local);
    else hipLaunchKernelGGL((k_small_mid<0>), dim3(1), dim3(threads), lds, s, p, nsteps, step_local);
    return hipGetLastError();
}

hipError_t launch_step(const StepParams &p, int dim, int prec, int mode, hipStream_t s, int step_local) {
    if (dim == 2) return prec ? launch_step_t<2, 1>(p, mode, s, step_local) : launch_step_t<2, 0>(p, mode, s, step_local);
    return prec ? launch_step_t<3, 1>(p, mode, s, step_local) : launch_step_t<3, 0>(p, mode, s, step_local);
}

template <int PREC, int POOL>
void launch_c3w(const StepParams &p, hipStream_t s, int step_local) {
    const dim3 grid(p.c_wblocks), block(kC3WinBlock);
    if (p.law == LSM_SPRING_RECOVER)
        hipLaunchKernelGGL((k_step_c3w<PREC, POOL, LSM_SPRING_RECOVER>), grid, block, 0, s, p, step_local);
    else if (p.law == LSM_SPRING_CUBIC)
        hipLaunchKernelGGL((k_step_c3w<PREC, POOL, LSM_SPRING_CUBIC>), grid, block, 0, s, p, step_local);
    else
        hipLaunchKernelGGL((k_step_c3w<PREC, POOL, LSM_SPRING_LINEAR>), grid, block, 0, s, p, step_local);
}

hipError_t launch_step_c3(const StepParams &p, int prec, hipStream_t s, int step_local, int kind) {
    const dim3 grid(p.c_blocks), block(kBlock);
    if (kind == 2) {
        if (prec) launch_c3w<1, kC3PoolF32>(p, s, step_local);
        else launch_c3w<0, kC3PoolF64>(p, s, step_local);
    } else if (kind == 1) {
        if (prec) hipLaunchKernelGGL((k_step_c3<1, true>), grid, block, 0, s, p, step_local);
        else hipLaunchKernelGGL((k_step_c3<0, true>), grid, block, 0, s, p, step_local);
    } else {
        if (prec) hipLaunchKernelGGL((k_step_c3<1, false>), grid, block, 0, s, p, step_local);
        else hipLaunchKernelGGL((k_step_c3<0, false>), grid, block, 0, s, p, step_local);
    }
    return hipGetLastError();
}

hipError_t launch_pack_c3(const StepParams &p, int prec, hipStream_t s, int to_compact, void *u_grid,
                          void *v_grid, uint32_t *m_grid, void *u_c, void *v_c, uint32_t *m_c, int64_t cn) {
    const uint32_t ncn = uint32_t(cn);
    const dim3 grid(unsigned((p.n_part + 255) / 256)), block(256);
    if (p.n_part <= 0) return hipSuccess;
    if (to_compact) {
        if (prec) hipLaunchKernelGGL((k_pack_c3<1, true>), grid, block, 0, s, p, u_grid, v_grid, m_grid, u_c, v_c, m_c, ncn);
        else hipLaunchKernelGGL((k_pack_c3<0, true>), grid, block, 0, s, p, u_grid, v_grid, m_grid, u_c, v_c, m_c, ncn);
    } else {
        if (prec) hipLaunchKernelGGL((k_pack_c3<1, false>), grid, block, 0, s, p, u_grid, v_grid, m_grid, u_c, v_c, m_c, ncn);
        else hipLaunchKernelGGL((k_pack_c3<0, false>), grid, block, 0, s, p, u_grid, v_grid, m_grid, u_c, v_c, m_c, ncn);
    }
    return hipGetLastError();
}

hipError_t launch_local_fields(const StepParams &p, int dim, int prec, hipStream_t s, const int32_t *site_of,
                               const int32_t *part_of, int radius, double vsite, double *stress, double *strain) {
    if (p.n_part <= 0) return hipSuccess;
    const dim3 grid(unsigned((p.n_part + 255) / 256)), block(256);
    // radius 1: the contributions go to `strain` first, which the strain
    // kernel then overwrites
    double *tmp = radius > 0 ? strain : stress;
    if (dim == 2) {
        if (prec) hipLaunchKernelGGL((k_virial<2, 1>), grid, block, 0, s, p, site_of, tmp);
        else hipLaunchKernelGGL((k_virial<2, 0>), grid, block, 0, s, p, site_of, tmp);
        hipLaunchKernelGGL((k_virial_domain<2>), grid, block, 0, s, p, site_of, part_of, tmp, stress, radius, vsite);
        if (prec) hipLaunchKernelGGL((k_strain<2, 1>), grid, block, 0, s, p, site_of, strain);
        else hipLaunchKernelGGL((k_strain<2, 0>), grid, block, 0, s, p, site_of, strain);
    } else {
        if (prec) hipLaunchKernelGGL((k_virial<3, 1>), grid, block, 0, s, p, site_of, tmp);
        else hipLaunchKernelGGL((k_virial<3, 0>), grid, block, 0, s, p, site_of, tmp);
        hipLaunchKernelGGL((k_virial_domain<3>), grid, block, 0, s, p, site_of, part_of, tmp, stress, radius, vsite);
        if (prec) hipLaunchKernelGGL((k_strain<3, 1>), grid, block, 0, s, p, site_of, strain);
        else hipLaunchKernelGGL((k_strain<3, 0>), grid, block, 0, s, p, site_of, strain);
    }
    return hipGetLastError();
}

hipError_t launch_increment(const StepParams &p, int dim, int prec, hipStream_t s, double eps_new,
                            double d_eps, int inc, int affine) {
    const dim3 grid(unsigned((p.nsites + 255) / 256)), block(256);
    if (dim == 2) {
        if (prec) hipLaunchKernelGGL((k_increment<2, 1>), grid, block, 0, s, p, eps_new, d_eps, inc, affine);
        else hipLaunchKernelGGL((k_increment<2, 0>), grid, block, 0, s, p, eps_new, d_eps, inc, affine);
    } else {
        if (prec) hipLaunchKernelGGL((k_increment<3, 1>), grid, block, 0, s, p, eps_new, d_eps, inc, affine);
        else hipLaunchKernelGGL((k_increment<3, 0>), grid, block, 0, s, p, eps_new, d_eps, inc, affine);
    }
    return hipGetLastError();
}

hipError_t launch_kick_drift(const StepParams &p, int dim, int prec, hipStream_t s) {
    const dim3 grid(unsigned((p.nsites + 255) / 256)), block(256);
    if (dim == 2) {
        if (prec) hipLaunchKernelGGL((k_kick_drift<2, 1>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_kick_drift<2, 0>), grid, block, 0, s, p);
    } else {
        if (prec) hipLaunchKernelGGL((k_kick_drift<3, 1>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_kick_drift<3, 0>), grid, block, 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_grips(const StepParams &p, int dim, int prec, hipStream_t s, int step_local) {
    const dim3 grid(unsigned((2 * int64_t(p.ny) * p.nz + 255) / 256)), block(256);
    if (dim == 2) {
        if (prec) hipLaunchKernelGGL((k_grips<2, 1>), grid, block, 0, s, p, step_local);
        else hipLaunchKernelGGL((k_grips<2, 0>), grid, block, 0, s, p, step_local);
    } else {
        if (prec) hipLaunchKernelGGL((k_grips<3, 1>), grid, block, 0, s, p, step_local);
        else hipLaunchKernelGGL((k_grips<3, 0>), grid, block, 0, s, p, step_local);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const StepParams &p, int dim, hipStream_t s, DevRecord *rec, double omega,
                           int nsteps) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, p, rec, omega, nsteps, dim);
    return hipGetLastError();
}

}  // namespace lsm
