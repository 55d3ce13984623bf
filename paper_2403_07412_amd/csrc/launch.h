// Launch machinery shared by the kernel translation units: the per-point
// conditional kernel, the implementation policies, variant selection and
// the launchers.  Each kernels_nu*.hip file instantiates the launchers for
// one smoothness, so the heavy kernels compile in parallel.
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
template <int NU, bool GRAD>
struct LdsImpl {
    static constexpr int NT = 256;
    static constexpr int WPE = 2;  // wavefronts per SIMD the register allocation targets
    static size_t smem(int m) { return lds_kernel_smem_bytes(m); }
    static __device__ CondOut run(const double *locs, const double *z, const int32_t *nbr, int64_t i, int32_t m,
                                  const Params &P, double *sm) {
        return lds_conditional<NU, GRAD>(locs, z, nbr, i, m, P, sm);
    }
};

template <int T, int W, int NU, bool GRAD>
struct TileImpl {
    static constexpr int NT = W * kWave;
    static constexpr int WPE = VECCHIA_WPE_OVERRIDE > 0 ? VECCHIA_WPE_OVERRIDE : tile_waves_per_simd(T, W);
    static size_t smem(int) { return TileLds<T>::BYTES; }
    static __device__ CondOut run(const double *locs, const double *z, const int32_t *nbr, int64_t i, int32_t m,
                                  const Params &P, double *sm) {
        return tile_conditional<T, W, NU, GRAD>(locs, z, nbr, i, m, P, sm);
    }
};

// One workgroup per listed point t (point i = idx[t], or t when idx is NULL).
// Writes l_i to ell[t * ell_stride] and the gradient to g[t * g_stride + 0..2]
// (NaN on failure), and reports failure through flags[t] (when given) or as
// atomicMin(status, t + 1) (when given).
template <class Impl>
__global__ void __launch_bounds__(Impl::NT) __attribute__((amdgpu_waves_per_eu(Impl::WPE)))
    cond_kernel(const double *__restrict__ locs, const double *__restrict__ z, const int32_t *__restrict__ nbr,
                int64_t n, int32_t m, const double *__restrict__ theta, const int64_t *__restrict__ idx,
                int64_t t0, double *__restrict__ ell, int64_t ell_stride, double *__restrict__ g,
                int64_t g_stride, int32_t *__restrict__ flags, unsigned long long *__restrict__ status) {
    extern __shared__ double smem[];
    const Params P = load_params(theta);
    const int64_t t = t0 + blockIdx.x;
    const int64_t i = idx ? idx[t] : t;
    CondOut o;
    bool bad = true;
    if (P.valid && i >= 0 && i < n) {  // uniform over the workgroup
        o = Impl::run(locs, z, nbr, i, m, P, smem);
        bad = o.bad;
    }
    if (bad) o.ell = o.g0 = o.g1 = o.g2 = __builtin_nan("");
    if (threadIdx.x == 0) {
        ell[t * ell_stride] = o.ell;
        if (g) {
            g[t * g_stride + 0] = o.g0;
            g[t * g_stride + 1] = o.g1;
            g[t * g_stride + 2] = o.g2;
        }
        if (flags) flags[t] = bad ? 1 : 0;
        if (status && bad && P.valid) atomicMin(status, (unsigned long long)(t + 1));
    }
}

template <typename K>
hipError_t allow_smem(K kernel, size_t bytes) {
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Arguments of one conditional-kernel launch.
struct EvalArgs {
    const double *locs, *z;
    const int32_t *nbr;
    int64_t n;
    int32_t m;
    const double *theta;
    const int64_t *idx;
    int64_t nidx;
    double *ell;
    int64_t ell_stride;
    double *g;
    int64_t g_stride;
    int32_t *flags;
    unsigned long long *status;
};

template <class Impl>
int launch_cond_impl(const EvalArgs &a, hipStream_t s) {
    if (a.nidx == 0) return VECCHIA_OK;
    const size_t smem = Impl::smem(a.m);
    auto kern = cond_kernel<Impl>;
    if (allow_smem(kern, smem) != hipSuccess) return VECCHIA_EHIP;
    constexpr int64_t kMaxGrid = (int64_t)1 << 22;  // blocks per launch; larger lists take several launches
    for (int64_t t0 = 0; t0 < a.nidx; t0 += kMaxGrid) {
        const int64_t grid = std::min<int64_t>(a.nidx - t0, kMaxGrid);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(Impl::NT), smem, s, a.locs, a.z, a.nbr, a.n, a.m, a.theta,
                           a.idx, t0, a.ell, a.ell_stride, a.g, a.g_stride, a.flags, a.status);
    }
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

// Kernel variants.  The tiled family is instantiated for T = ceil((m+2)/16)
// tile rows and W wavefronts per conditional.
enum Variant { V_AUTO = 0, V_UNBLOCKED = 1, V_TILE_W1 = 2, V_TILE_W2 = 3, V_TILE_W4 = 4, V_TILE_W8 = 5 };

constexpr int kMaxT = (VECCHIA_MAX_M + 2 + 15) / 16;

inline int tile_rows(int m) { return (m + 2 + 15) / 16; }

// register budget: at most 20 tiles per wavefront
inline bool variant_feasible(int variant, int m) {
    if (variant == V_UNBLOCKED) return true;
    const int T = tile_rows(m);
    const int W = variant == V_TILE_W1 ? 1 : variant == V_TILE_W2 ? 2 : variant == V_TILE_W4 ? 4 : 8;
    if (W > 1 && tile_count(T) < W) return false;
    return tiles_per_wave(T, W) <= 20;
}

inline int default_variant(int m) {
    const int T = tile_rows(m);
    if (T <= 2) return V_TILE_W1;
    if (T <= 4) return V_TILE_W2;
    if (T <= 8) return V_TILE_W4;
    return V_TILE_W8;
}

template <int NU, bool GRAD, int T, int W>
int launch_tile(const EvalArgs &a, hipStream_t s) {
    if constexpr (W > 1 && tile_count(T) < W) {
        return VECCHIA_EUNSUPPORTED;
    } else if constexpr (tiles_per_wave(T, W) > 20) {
        return VECCHIA_EUNSUPPORTED;
    } else {
        return launch_cond_impl<TileImpl<T, W, NU, GRAD>>(a, s);
    }
}

template <int NU, bool GRAD, int W>
int launch_tile_w(int T, const EvalArgs &a, hipStream_t s) {
#ifdef VECCHIA_ONE_VARIANT
    if (T == 8 && W == 4) return launch_tile<NU, GRAD, 8, 4>(a, s);
    return VECCHIA_EUNSUPPORTED;
#else
    switch (T) {
        case 1: return launch_tile<NU, GRAD, 1, W>(a, s);
        case 2: return launch_tile<NU, GRAD, 2, W>(a, s);
        case 3: return launch_tile<NU, GRAD, 3, W>(a, s);
        case 4: return launch_tile<NU, GRAD, 4, W>(a, s);
        case 5: return launch_tile<NU, GRAD, 5, W>(a, s);
        case 6: return launch_tile<NU, GRAD, 6, W>(a, s);
        case 7: return launch_tile<NU, GRAD, 7, W>(a, s);
        case 8: return launch_tile<NU, GRAD, 8, W>(a, s);
        case 9: return launch_tile<NU, GRAD, 9, W>(a, s);
        case 10: return launch_tile<NU, GRAD, 10, W>(a, s);
        case 11: return launch_tile<NU, GRAD, 11, W>(a, s);
        default: return VECCHIA_EUNSUPPORTED;
    }
#endif
}

template <int NU, bool GRAD>
int launch_variant(int variant, const EvalArgs &a, hipStream_t s) {
    const int T = tile_rows(a.m);
    switch (variant) {
        case V_UNBLOCKED:
            return launch_cond_impl<LdsImpl<NU, GRAD>>(a, s);
        case V_TILE_W1: return launch_tile_w<NU, GRAD, 1>(T, a, s);
        case V_TILE_W2: return launch_tile_w<NU, GRAD, 2>(T, a, s);
        case V_TILE_W4: return launch_tile_w<NU, GRAD, 4>(T, a, s);
        case V_TILE_W8: return launch_tile_w<NU, GRAD, 8>(T, a, s);
        default: return VECCHIA_EUNSUPPORTED;
    }
}

// Defined in kernels_nu05.hip, kernels_nu15.hip and kernels_nu25.hip.
int launch_nu05(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_nu15(bool grad, int variant, const EvalArgs &a, hipStream_t s);
int launch_nu25(bool grad, int variant, const EvalArgs &a, hipStream_t s);

}  // namespace vecchia
