// Launch machinery shared by the kernel translation units: the per-point
// conditional kernel, the implementation policies, variant selection and
// the launchers.  Each kernels_*.hip file instantiates the launchers for one
// covariance code (Matern smoothness or power exponential, with Euclidean or
// great-circle distance), so the heavy kernels compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "kernel_lds.h"
#include "kernel_tile.h"
#include "vecchia.h"

#ifndef VECCHIA_WPE_OVERRIDE
#define VECCHIA_WPE_OVERRIDE 0
#endif

namespace vecchia {

// Implementation policies: how one conditional is evaluated by a workgroup.
template <int KC, bool GRAD>
struct LdsImpl {
    static constexpr int NT = 256;
    static constexpr int WPE = 2;  // wavefronts per SIMD the register allocation targets
    static size_t smem(int m) { return lds_kernel_smem_bytes(m); }
    static __device__ CondOut run(const double *locs, const double *z, const int32_t *nbr, int64_t i, int64_t n,
                                  int32_t m, const double *qloc, const Params &P, double *sm) {
        return lds_conditional<KC, GRAD>(locs, z, nbr, i, n, m, qloc, P, sm);
    }
};

// G > 1: G parameter vectors of one conditional per workgroup (lockstep).
template <int T, int W, int KC, bool GRAD, int G = 1>
struct TileImpl {
    static constexpr int NT = G * W * kWave;
    static constexpr int GROUP = G;
    static constexpr int WAVES = W;  // wavefronts per parameter vector
    static constexpr bool GCD = kc_gcd(KC);
    static constexpr int WPE = VECCHIA_WPE_OVERRIDE > 0
                                   ? VECCHIA_WPE_OVERRIDE
                                   : tile_waves_per_simd(T, W, GRAD && keep_dbeta(T, W, GCD), GRAD, GCD, G);
    static size_t smem(int) { return TileLds<T, W, GRAD, GCD, G>::BYTES; }
    static __device__ CondOut run(const double *locs, const double *z, const int32_t *nbr, int64_t i, int64_t n,
                                  int32_t m, const double *qloc, const Params &P, double *sm) {
        return tile_conditional<T, W, KC, GRAD, G>(locs, z, nbr, i, n, m, qloc, P, sm);
    }
};

// A field of a batched evaluation, as the device sees it (a table the
// batched entry points write into the caller's workspace).
struct FieldDev {
    const double *locs;   // [n][2]
    const double *z;      // [n]
    const int32_t *nbr;   // [n][m]
    int64_t n;
    int64_t m;
    int64_t eval0;        // evaluation index of (this field, theta 0); evaluation e = field * ntheta + theta
    int64_t vals0;        // row of (this field, theta 0, point 0) in the per-point value array
    int64_t pb0;          // first reduce block of (this field, theta 0); theta q owns [pb0 + q nb, + nb)
    int64_t nb;           // reduce blocks per evaluation of this field
};

// Arguments of one conditional-kernel launch (passed by value).
//   single mode (fields == NULL): item t is point idx[t] (or t) of one field;
//     results go to row t - row0 of ell (ell[row * ell_stride]), g
//     (g[row * g_stride + 0..2]) and flags, or to status;
//   batched mode: the items of a tile class, t in [0, item0[nfc]); item t lies
//     in class field c (item0[c] <= t < item0[c+1]) = fields[fidx[c]]; with
//     r = t - item0[c], the point is i = n - 1 - r / ntheta (items run from the
//     last point, whose conditioning set is full, to the first) and the theta
//     index q = r % ntheta; results go to row vals0 + q n + i of ell / g /
//     flags, parameters come from theta + 3 (eval0 + q);
//   prediction mode (qlocs != NULL, single mode only): item t is prediction
//     point t < nq at qlocs[t], conditioned on row t of nbr among the n
//     points of locs / z; mean and variance go to pmean[t], pvar[t].
// alpha is the power-exponential exponent (ignored by the Matern codes).
struct KernelArgs {
    const double *locs, *z;
    const int32_t *nbr;
    int64_t n;
    int32_t m;
    const double *theta;
    const int64_t *idx;
    const FieldDev *fields;
    const int32_t *fidx;
    const int64_t *item0;
    int32_t nfc;
    int32_t ntheta;
    double *ell;
    int64_t ell_stride;
    double *g;
    int64_t g_stride;
    int32_t *flags;
    unsigned long long *status;
    int64_t t0;
    int64_t row0;  // single mode: results of item t go to row t - row0
    double alpha;
    const double *qlocs;
    int64_t nq;
    double *pmean, *pvar;
};

// r / ntheta for an item offset r >= 0 of the lockstep form: in 32 bits when
// r fits (a 64-bit division is a long instruction sequence at the start of
// every workgroup).  The one-vector form keeps the plain division: the
// branch costs the m = 120 kernel a scalar spill.
__device__ __forceinline__ int64_t item_point(int64_t r, int32_t ntheta) {
    if (ntheta == 1) return r;
    if ((r >> 32) == 0) return (int64_t)((uint32_t)r / (uint32_t)ntheta);
    return r / ntheta;
}

// Evaluates item t (see KernelArgs) with one workgroup.  Failure is reported
// through flags[row] (when given) or as atomicMin(status, t + 1) (when
// given); failed rows hold NaN.
template <class Impl>
__device__ __forceinline__ void cond_item(const KernelArgs &a, int64_t t, double *smem) {
    const double *locs = a.locs, *z = a.z, *theta = a.theta;
    const int32_t *nbr = a.nbr;
    int64_t n = a.n, i, row;
    int32_t m = a.m;
    if (a.fields) {
        int lo = 0, hi = a.nfc;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.item0[mid] <= t) lo = mid;
            else hi = mid;
        }
        const FieldDev &F = a.fields[a.fidx[lo]];
        locs = F.locs;
        z = F.z;
        nbr = F.nbr;
        n = F.n;
        m = (int32_t)F.m;
        const int64_t r = t - a.item0[lo];
        const int64_t ip = r / a.ntheta;
        const int64_t q = r - ip * a.ntheta;
        i = n - 1 - ip;
        theta = a.theta + 3 * (F.eval0 + q);
        row = F.vals0 + q * n + i;
    } else {
        i = a.idx ? a.idx[t] : t;
        row = t - a.row0;
    }
    const Params P = load_params(theta, a.alpha);
    const bool pred = a.qlocs != nullptr;
    const int64_t nitems = pred ? a.nq : n;
    CondOut o;
    bool bad = true;
    if (P.valid && i >= 0 && i < nitems) {  // uniform over the workgroup
        o = Impl::run(locs, z, nbr, i, n, m, pred ? a.qlocs + 2 * i : nullptr, P, smem);
        bad = o.bad;
    }
    if (bad) o.ell = o.g0 = o.g1 = o.g2 = o.mean = o.var = __builtin_nan("");
    if (threadIdx.x == 0) {
        if (pred) {
            a.pmean[row] = o.mean;
            a.pvar[row] = o.var;
        } else {
            a.ell[row * a.ell_stride] = o.ell;
        }
        if (a.g) {
            a.g[row * a.g_stride + 0] = o.g0;
            a.g[row * a.g_stride + 1] = o.g1;
            a.g[row * a.g_stride + 2] = o.g2;
        }
        if (a.flags) a.flags[row] = bad ? 1 : 0;
        if (a.status && bad && P.valid) atomicMin(a.status, (unsigned long long)(t + 1));
    }
}

// One workgroup per item.  (A persistent form, workgroups pulling items from
// a counter, kept about 25 more VGPRs and twice the scalar spills live across
// its loop in the T = 8, W = 4 kernel, one workgroup per CU less: slower.)
template <class Impl>
__global__ void __launch_bounds__(Impl::NT) __attribute__((amdgpu_waves_per_eu(Impl::WPE)))
    cond_kernel(const KernelArgs a) {
    extern __shared__ double smem[];
    cond_item<Impl>(a, a.t0 + blockIdx.x, smem);
}

template <typename K>
hipError_t allow_smem(K kernel, size_t bytes) {
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Batched mode, lockstep form: the G wavefront groups of a workgroup take the
// G consecutive items t, t + 1, .., t + G - 1 (t a multiple of G), which are
// the same point of one field for G consecutive parameter vectors because
// ntheta is a multiple of G.  Each group loads its own parameters; a group
// whose vector is invalid runs on placeholder parameters (the workgroup's
// barriers need every group) and reports its row as failed.
template <class Impl>
__device__ __forceinline__ void cond_item_group(const KernelArgs &a, int64_t t0, double *smem) {
    constexpr int G = Impl::GROUP;
    const int wq = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)) / Impl::WAVES;
    const int64_t t = t0 + wq;
    int lo = 0, hi = a.nfc;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.item0[mid] <= t) lo = mid;
        else hi = mid;
    }
    const FieldDev &F = a.fields[a.fidx[lo]];
    const int64_t r = t - a.item0[lo];
    const int64_t ip = item_point(r, a.ntheta);
    const int64_t q = r - ip * a.ntheta;
    const int64_t n = F.n, i = n - 1 - ip;
    const int64_t row = F.vals0 + q * n + i;
    Params P = load_params(a.theta + 3 * (F.eval0 + q), a.alpha);
    const bool valid = P.valid;
    if (!valid) {
        P.sigma2 = 1.0;
        P.beta = 1.0;
        P.inv_beta = 1.0;
        P.tau2 = 1.0;
    }
    static_assert(G > 1, "the lockstep form");
    CondOut o = Impl::run(F.locs, F.z, F.nbr, i, n, (int32_t)F.m, nullptr, P, smem);
    const bool bad = o.bad || !valid;
    if (bad) o.ell = o.g0 = o.g1 = o.g2 = __builtin_nan("");
    if (threadIdx.x % (Impl::WAVES * kWave) == 0) {
        a.ell[row * a.ell_stride] = o.ell;
        if (a.g) {
            a.g[row * a.g_stride + 0] = o.g0;
            a.g[row * a.g_stride + 1] = o.g1;
            a.g[row * a.g_stride + 2] = o.g2;
        }
        if (a.flags) a.flags[row] = bad ? 1 : 0;
        if (a.status && bad && valid) atomicMin(a.status, (unsigned long long)(t + 1));
    }
}

template <class Impl>
__global__ void __launch_bounds__(Impl::NT) __attribute__((amdgpu_waves_per_eu(Impl::WPE)))
    cond_group_kernel(const KernelArgs a) {
    extern __shared__ double smem[];
    cond_item_group<Impl>(a, a.t0 + (int64_t)Impl::GROUP * blockIdx.x, smem);
}

// A launch request: kernel arguments plus the item range [t_begin, t_end)
// and the largest m among the items (sizes the LDS of the unblocked kernel).
// group > 1 asks for the lockstep form with that many parameter vectors per
// workgroup (batched mode; the range and ntheta are multiples of it).
struct EvalArgs {
    KernelArgs k;
    int64_t t_begin, t_end;
    int32_t m_max;
    int32_t group;
};

template <class Impl>
int launch_cond_impl(const EvalArgs &a, hipStream_t s) {
    if (a.t_end <= a.t_begin) return VECCHIA_OK;
    const size_t smem = Impl::smem(a.m_max);
    auto kern = cond_kernel<Impl>;
    if (allow_smem(kern, smem) != hipSuccess) return VECCHIA_EHIP;
    constexpr int64_t kMaxGrid = (int64_t)1 << 22;  // workgroups per launch; longer ranges take several launches
    for (int64_t t0 = a.t_begin; t0 < a.t_end; t0 += kMaxGrid) {
        const int64_t grid = std::min<int64_t>(a.t_end - t0, kMaxGrid);
        KernelArgs k = a.k;
        k.t0 = t0;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(Impl::NT), smem, s, k);
    }
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

template <class Impl>
int launch_group_impl(const EvalArgs &a, hipStream_t s) {
    constexpr int G = Impl::GROUP;
    if (a.t_end <= a.t_begin) return VECCHIA_OK;
    if (!a.k.fields || a.k.qlocs || a.k.ntheta % G != 0 || a.t_begin % G != 0 || a.t_end % G != 0)
        return VECCHIA_EINVAL;
    const size_t smem = Impl::smem(a.m_max);
    auto kern = cond_group_kernel<Impl>;
    if (allow_smem(kern, smem) != hipSuccess) return VECCHIA_EHIP;
    constexpr int64_t kMaxGrid = (int64_t)1 << 22;
    for (int64_t t0 = a.t_begin; t0 < a.t_end; t0 += kMaxGrid * G) {
        const int64_t grid = std::min<int64_t>((a.t_end - t0) / G, kMaxGrid);
        KernelArgs k = a.k;
        k.t0 = t0;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(Impl::NT), smem, s, k);
    }
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

// Kernel variants.  The tiled family is instantiated for T = ceil((m+2)/16)
// tile rows and W wavefronts per conditional.
enum Variant { V_AUTO = 0, V_UNBLOCKED = 1, V_TILE_W1 = 2, V_TILE_W2 = 3, V_TILE_W4 = 4, V_TILE_W8 = 5 };

constexpr int kMaxT = (VECCHIA_MAX_M + 2 + 15) / 16;

inline int tile_rows(int m) { return (m + 2 + 15) / 16; }

// wavefronts per conditional of a tiled variant (0 for the unblocked kernel)
inline int variant_waves(int variant) {
    switch (variant) {
        case V_TILE_W1: return 1;
        case V_TILE_W2: return 2;
        case V_TILE_W4: return 4;
        case V_TILE_W8: return 8;
        default: return 0;
    }
}

// register budget: at most 20 tiles per wavefront
inline bool variant_feasible(int variant, int m) {
    if (variant == V_UNBLOCKED) return true;
    const int T = tile_rows(m);
    const int W = variant == V_TILE_W1 ? 1 : variant == V_TILE_W2 ? 2 : variant == V_TILE_W4 ? 4 : 8;
    if (W > 1 && tile_count(T) < W) return false;
    return tiles_per_wave(T, W) <= 20;
}

// Built-in choice when the variant table has no entry: the fastest variant
// per tile count measured on MI355X (value and value + gradient, nu = 1/2,
// 3/2, 5/2, 60,000 uniform points; rows 4 with the gradient re-measured at
// 300,000 points, nu = 1/2, once the occupancy targets allowed a fifth
// wavefront per SIMD).  Three and four tile rows favour one wavefront with
// the gradient and two without; up to six rows two wavefronts; beyond, four
// (eight wavefronts lose to their barriers at every size).  Since the
// one-wavefront kernels factor their diagonal tiles in place, one wavefront
// is also the faster value-only kernel at three and four rows for the Matern
// codes on Euclidean distances (kc 0..2; 250,000 points: 1.56 against 1.77 ms
// at m = 40, 2.78 against 2.83 ms at m = 60), but not for kriging with the
// great-circle power exponential (25,000 predictions at m = 60: 0.84 against
// 0.69 ms): the other codes, kriging (kc < 0) and unknown callers keep two.
inline int default_variant(int m, bool grad, int kc = -1) {
    const int T = tile_rows(m);
    if (T <= 2) return V_TILE_W1;
    if (T <= 4) return (grad || (kc >= 0 && kc <= 2)) ? V_TILE_W1 : V_TILE_W2;
    if (T <= 6) return V_TILE_W2;
    return V_TILE_W4;
}

template <int KC, bool GRAD, int T, int W>
int launch_tile(const EvalArgs &a, hipStream_t s) {
    if constexpr (W > 1 && tile_count(T) < W) {
        return VECCHIA_EUNSUPPORTED;
    } else if constexpr (tiles_per_wave(T, W) > 20) {
        return VECCHIA_EUNSUPPORTED;
    } else {
        constexpr int G = lockstep_group(T, W);
        if (a.group > 1) {
            if constexpr (G > 1) {
                if (a.group == G) return launch_group_impl<TileImpl<T, W, KC, GRAD, G>>(a, s);
            }
            return VECCHIA_EUNSUPPORTED;
        }
        return launch_cond_impl<TileImpl<T, W, KC, GRAD>>(a, s);
    }
}

template <int KC, bool GRAD, int W>
int launch_tile_w(int T, const EvalArgs &a, hipStream_t s) {
#ifdef VECCHIA_ONE_VARIANT
    if (T == 8 && W == 4) return launch_tile<KC, GRAD, 8, 4>(a, s);
    return VECCHIA_EUNSUPPORTED;
#else
    switch (T) {
        case 1: return launch_tile<KC, GRAD, 1, W>(a, s);
        case 2: return launch_tile<KC, GRAD, 2, W>(a, s);
        case 3: return launch_tile<KC, GRAD, 3, W>(a, s);
        case 4: return launch_tile<KC, GRAD, 4, W>(a, s);
        case 5: return launch_tile<KC, GRAD, 5, W>(a, s);
        case 6: return launch_tile<KC, GRAD, 6, W>(a, s);
        case 7: return launch_tile<KC, GRAD, 7, W>(a, s);
        case 8: return launch_tile<KC, GRAD, 8, W>(a, s);
        case 9: return launch_tile<KC, GRAD, 9, W>(a, s);
        case 10: return launch_tile<KC, GRAD, 10, W>(a, s);
        case 11: return launch_tile<KC, GRAD, 11, W>(a, s);
        default: return VECCHIA_EUNSUPPORTED;
    }
#endif
}

template <int KC, bool GRAD>
int launch_variant(int variant, const EvalArgs &a, hipStream_t s) {
    const int T = tile_rows(a.m_max);
    switch (variant) {
        case V_UNBLOCKED:
            if (a.group > 1) return VECCHIA_EUNSUPPORTED;
            return launch_cond_impl<LdsImpl<KC, GRAD>>(a, s);
        case V_TILE_W1: return launch_tile_w<KC, GRAD, 1>(T, a, s);
        case V_TILE_W2: return launch_tile_w<KC, GRAD, 2>(T, a, s);
        case V_TILE_W4: return launch_tile_w<KC, GRAD, 4>(T, a, s);
        case V_TILE_W8: return launch_tile_w<KC, GRAD, 8>(T, a, s);
        default: return VECCHIA_EUNSUPPORTED;
    }
}

// Defined in vecchia.hip: smoothness code (0, 1, 2 for nu = 0.5, 1.5, 2.5;
// -1 otherwise), the variant a launch uses for (m, gradient), the host-side
// variant table, and the launcher for any covariance code (0..7).
int nu_code(double nu);
int cov_code(const vecchia_cov *cov, double *alpha);
int resolve_variant(int m, bool grad, int requested, int kc = -1);
extern int g_variant[2][VECCHIA_MAX_M + 1];
int launch_any(int kc, bool grad, int variant, const EvalArgs &a, hipStream_t s);

// Defined in kernels_nu05.hip, kernels_nu15.hip, kernels_nu25.hip (Matern,
// Euclidean) and kernels_kc3.hip .. kernels_kc7.hip (the other codes).
int launch_nu05(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_nu15(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_nu25(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_kc3(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_kc4(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_kc5(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_kc6(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_kc7(bool grad, int variant, const EvalArgs &a, hipStream_t s);

}  // namespace vecchia
