// Rasterisation stage: camera transform, perspective projection, clipping and
// colour, fused into one pass over the particle arrays (Sect. 2.1 and
// Sect. 3.1 describe transform and colour as per-particle loops; Sect. 4.3
// notes the GPU version fused them so inactive particles leave early).
//
// One thread per particle, grid-stride, coalesced structure-of-arrays loads.
// Position arithmetic runs in FP64 so the single-precision record keeps the
// screen position as integer part + fraction.  The colour map lookup and the
// peak amplitude 1/(pi sigma^2) (from the stored sigma) run in FP32.  A
// species coloured from the vector field takes the particle's own RGB instead
// of the colour map (Sect. 2.1 allows either).  Output
// per active particle: a 32-byte record, optionally the 8-byte sorted-mode
// record, and the 8-byte tile span read by the binning kernels.
#include "bin_device.h"

namespace spl {

namespace {

// kDt: the stored attribute type (SPL_F32, SPL_BF16 or SPL_F16), fixed per
// kernel instance so that the loads need no branch.
template <int kDt>
__device__ __forceinline__ float load_attr_t(const void *p, int64_t i) {
  if (kDt == SPL_F32) return static_cast<const float *>(p)[i];
  if (kDt == SPL_BF16) {
    const uint32_t b = static_cast<const uint16_t *>(p)[i];
    return __uint_as_float(b << 16);
  }
  return (float)static_cast<const _Float16 *>(p)[i];
}

__device__ __forceinline__ float load_attr(const void *p, int dtype, int64_t i) {
  if (dtype == SPL_F32) return static_cast<const float *>(p)[i];
  if (dtype == SPL_BF16) {
    const uint32_t b = static_cast<const uint16_t *>(p)[i];
    return __uint_as_float(b << 16);
  }
  return (float)static_cast<const _Float16 *>(p)[i];
}

__device__ __forceinline__ bool finitef(float v) { return __builtin_isfinite(v); }

// kCount: the tile counts of the binning stage are accumulated here too, in
// an LDS histogram per workgroup flushed once at the end, which saves a pass
// over the spans.
template <bool kCount, int kDt>
__global__ __launch_bounds__(kBlock) void k_project(ProjK P, TileK tk, float4 *__restrict__ rec,
                                                    float2 *__restrict__ rec2,
                                                    uint2 *__restrict__ span, int write_inactive,
                                                    Totals *__restrict__ tot,
                                                    uint32_t *__restrict__ counts) {
  extern __shared__ uint32_t hist[];
  __shared__ unsigned int s_act, s_large;
  // the species' looks, read per lane (the species select would otherwise
  // keep every look in scalar registers)
  __shared__ LookK s_looks[SPL_MAX_SPECIES];
  const int nb = tk.n_tiles + tk.n_ctiles;
  if (threadIdx.x == 0) {
    s_act = 0;
    s_large = 0;
  }
  if (threadIdx.x < SPL_MAX_SPECIES) s_looks[threadIdx.x] = P.looks[threadIdx.x];
  if (kCount)
    for (int i = threadIdx.x; i < nb; i += kBlock) hist[i] = 0;
  __syncthreads();
  unsigned int my_act = 0, my_large = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  // uniform trip count: the counting helpers need every lane of the wave
  for (int64_t kb = (int64_t)blockIdx.x * kBlock; kb < P.n; kb += stride) {
    const int64_t k = kb + threadIdx.x;
    uint2 spn = make_uint2(kInactive, kInactive);
    if (k < P.n) {
      const float x = P.x[k], y = P.y[k], z = P.z[k];
      const float h = load_attr_t<kDt>(P.h, k) * P.h_scale;
      const float I = load_attr_t<kDt>(P.inten, k) * P.i_scale;
      const float s = load_attr_t<kDt>(P.scal, k) * P.s_scale;
      const int sp = P.species ? (int)P.species[k] : 0;
      const float a = (P.mode == SPL_SORTED) ? P.absorb[k] : 0.0f;
      // Straight-line form: every lane computes the record and the tests
      // decide at the end whether it is kept (nested early exits would make
      // the compiler re-zero the outputs on every level of the main path).
      const bool in_ok = finitef(x) && finitef(y) && finitef(z) && finitef(h) && finitef(I) &&
                         finitef(s) && finitef(a) && h > 0.0f && a >= 0.0f && sp < P.n_species;
      const double vx = (double)x - P.e[0], vy = (double)y - P.e[1], vz = (double)z - P.e[2];
      const double zv = vx * P.f[0] + vy * P.f[1] + vz * P.f[2];
      const double xv = vx * P.r[0] + vy * P.r[1] + vz * P.r[2];
      const double yv = vx * P.u[0] + vy * P.u[1] + vz * P.u[2];
      // 1/zv: hardware reciprocal and two Newton steps (used when zv > z_near > 0)
      double iz = __builtin_amdgcn_rcp(zv);
      iz = fma(iz, fma(-zv, iz, 1.0), iz);
      iz = fma(iz, fma(-zv, iz, 1.0), iz);
      const double X = P.cx + P.F * xv * iz;
      const double Y = P.cy - P.F * yv * iz;
      const double rho = P.F * (double)h * iz;
      const double ks = P.k_sigma * rho;
      const double sig = sqrt(ks * ks + P.sigma_min * P.sigma_min);
      const double R = P.nu * sig;
      const bool in_view = in_ok && zv > P.z_near && fabs(X - P.cx) <= 4194304.0 &&
                           fabs(Y - P.cy) <= 4194304.0 && R <= 4194304.0;
      const LookK L = s_looks[in_ok ? sp : 0];
      float c0, c1, c2;
      bool colour_ok = true;
      if (L.vec) {
        // colour taken directly from the vector field
        c0 = c1 = c2 = 0.0f;
        if (in_view) {
          c0 = load_attr_t<kDt>(P.rgb, 3 * k) * P.c_scale;
          c1 = load_attr_t<kDt>(P.rgb, 3 * k + 1) * P.c_scale;
          c2 = load_attr_t<kDt>(P.rgb, 3 * k + 2) * P.c_scale;
        }
        colour_ok = finitef(c0) && finitef(c1) && finitef(c2);
      } else if (L.M == 1) {
        c0 = L.rgb[0];
        c1 = L.rgb[1];
        c2 = L.rgb[2];
      } else {
        float t;
        if (L.log10)
          t = (s > 0.0f) ? (log10f(s) - L.lo) * L.inv_range : 0.0f;
        else
          t = (s - L.lo) * L.inv_range;
        t = fminf(fmaxf(t, 0.0f), 1.0f);
        const float u = t * (float)(L.M - 1);
        int j = (int)floorf(u);
        j = min(max(j, 0), L.M - 2);
        const float fr = u - (float)j;
        const float *p0 = L.rgb + 3 * j;
        c0 = (1.0f - fr) * p0[0] + fr * p0[3];
        c1 = (1.0f - fr) * p0[1] + fr * p0[4];
        c2 = (1.0f - fr) * p0[2] + fr * p0[5];
      }
      const float bi = L.beta * I;
      const float E0 = bi * c0, E1 = bi * c1, E2 = bi * c2;
      const bool emits = (E0 != 0.0f) || (E1 != 0.0f) || (E2 != 0.0f);
      const bool keep = in_view && colour_ok && (emits || (P.mode == SPL_SORTED && a > 0.0f));
      // peak amplitude 1/(pi sigma^2) in single precision from the stored sigma
      const float sg = (float)sig;
      const float amp = __builtin_amdgcn_rcpf(3.14159265f * sg * sg);
      const double fX = floor(X), fY = floor(Y);
      float4 o0 = make_float4((float)fX, (float)(X - fX), (float)fY, (float)(Y - fY));
      float4 o1 = make_float4(sg, E0 * amp, E1 * amp, E2 * amp);
      float2 o2 = make_float2(a * amp, (float)zv);
      if (keep) spn = record_span(o0, o1.x, tk);
      const bool active = spn.x != kInactive;
      if (active) {
        ++my_act;
        if (spn.y & kLargeFlag) ++my_large;
      }
      if (active || write_inactive) {
        if (!active) {
          o0 = make_float4(0.f, 0.f, 0.f, 0.f);
          o1 = o0;
          o2 = make_float2(0.f, 0.f);
        }
        rec[2 * k] = o0;
        rec[2 * k + 1] = o1;
        if (rec2) rec2[k] = o2;
      }
      span[k] = spn;
    }
    // every lane of the wave takes part
    if (kCount) count_span(spn, k, rec, tk, hist);
  }
  if (kCount) {
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kBlock) {
      const uint32_t v = hist[i];
      if (v) atomicAdd(&counts[i], v);
    }
  }
  if (my_act) atomicAdd(&s_act, my_act);
  if (my_large) atomicAdd(&s_large, my_large);
  __syncthreads();
  if (threadIdx.x == 0 && tot) {
    if (s_act) atomicAdd(&tot->n_active, (unsigned long long)s_act);
    if (s_large) atomicAdd(&tot->n_large, (unsigned long long)s_large);
  }
}

__global__ __launch_bounds__(kBlock) void k_span_from_records(const float4 *__restrict__ rec,
                                                              int64_t n, TileK tk,
                                                              uint2 *__restrict__ span,
                                                              Totals *__restrict__ tot) {
  __shared__ unsigned int s_act;
  if (threadIdx.x == 0) s_act = 0;
  __syncthreads();
  unsigned int my_act = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
    const float4 r0 = rec[2 * k];
    const float4 r1 = rec[2 * k + 1];
    const uint2 sp = record_span(r0, r1.x, tk);
    span[k] = sp;
    if (sp.x != kInactive) ++my_act;
  }
  if (my_act) atomicAdd(&s_act, my_act);
  __syncthreads();
  if (threadIdx.x == 0 && s_act) atomicAdd(&tot->n_active, (unsigned long long)s_act);
}

// Order-preserving map of a double onto unsigned 64-bit keys, so that atomic
// integer min / max give the floating-point min / max exactly.
__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(kBlock) void k_scalar_range(ProjK P, int n_species, int log10s,
                                                         unsigned long long *__restrict__ mm) {
  __shared__ unsigned long long s_mm[2 * SPL_MAX_SPECIES];
  if (threadIdx.x < 2 * SPL_MAX_SPECIES)
    s_mm[threadIdx.x] = (threadIdx.x & 1) ? 0ull : ~0ull;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < P.n; k += stride) {
    const float s = load_attr(P.scal, P.dtype, k) * P.s_scale;
    const int sp = P.species ? (int)P.species[k] : 0;
    if (sp >= n_species || !finitef(s)) continue;
    double g = (double)s;
    if (log10s) {
      if (!(s > 0.0f)) continue;
      g = log10(g);
    }
    const unsigned long long key = order_key(g);
    atomicMin(&s_mm[2 * sp], key);
    atomicMax(&s_mm[2 * sp + 1], key);
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * n_species) {
    const unsigned long long v = s_mm[threadIdx.x];
    if (threadIdx.x & 1) {
      if (v != 0ull) atomicMax(&mm[threadIdx.x], v);
    } else {
      if (v != ~0ull) atomicMin(&mm[threadIdx.x], v);
    }
  }
}

__global__ void k_init_minmax(unsigned long long *mm, int n) {
  const int i = threadIdx.x;
  if (i < 2 * n) mm[i] = (i & 1) ? 0ull : ~0ull;
}

__global__ void k_decode_minmax(const unsigned long long *mm, int n, double *out) {
  const int i = threadIdx.x;
  if (i < 2 * n) {
    const unsigned long long k = mm[i];
    double v;
    if ((i & 1) ? (k == 0ull) : (k == ~0ull)) {
      v = (i & 1) ? -__builtin_inf() : __builtin_inf();
    } else {
      const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
      v = __longlong_as_double((long long)b);
    }
    out[i] = v;
  }
}

int grid_for(int64_t n, int per_block_items, int max_blocks) {
  int64_t g = (n + per_block_items - 1) / per_block_items;
  if (g < 1) g = 1;
  if (g > max_blocks) g = max_blocks;
  return (int)g;
}

}  // namespace

bool project_counts(const TileK &tk) { return tk.n_tiles + tk.n_ctiles <= kProjectBins; }

hipError_t launch_project(const ProjK &pk, const TileK &tk, float *rec, float *rec2, uint2 *span,
                          int write_inactive, Totals *tot, hipStream_t s, uint32_t *counts) {
  if (pk.n == 0) return hipSuccess;
  auto launch = [&](auto kernel, int g, size_t sh, uint32_t *cnt) {
    hipLaunchKernelGGL(kernel, dim3(g), dim3(kBlock), sh, s, pk, tk,
                       reinterpret_cast<float4 *>(rec), reinterpret_cast<float2 *>(rec2), span,
                       write_inactive, tot, cnt);
  };
  if (counts && project_counts(tk)) {
    // fewer, longer-lived workgroups: each flushes its histogram once
    const int g = grid_for(pk.n, kBlock, 4096);
    const size_t sh = (size_t)(tk.n_tiles + tk.n_ctiles) * sizeof(uint32_t);
    if (pk.dtype == SPL_BF16)
      launch(k_project<true, SPL_BF16>, g, sh, counts);
    else if (pk.dtype == SPL_F16)
      launch(k_project<true, SPL_F16>, g, sh, counts);
    else
      launch(k_project<true, SPL_F32>, g, sh, counts);
  } else {
    const int g = grid_for(pk.n, kBlock, 8192);
    if (pk.dtype == SPL_BF16)
      launch(k_project<false, SPL_BF16>, g, 0, nullptr);
    else if (pk.dtype == SPL_F16)
      launch(k_project<false, SPL_F16>, g, 0, nullptr);
    else
      launch(k_project<false, SPL_F32>, g, 0, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_span_from_records(const float *rec, int64_t n, const TileK &tk, uint2 *span,
                                    Totals *tot, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int g = grid_for(n, kBlock, 8192);
  hipLaunchKernelGGL(k_span_from_records, dim3(g), dim3(kBlock), 0, s,
                     reinterpret_cast<const float4 *>(rec), n, tk, span, tot);
  return hipGetLastError();
}

// out_minmax: device buffer of 2 * SPL_MAX_SPECIES u64 keys followed by
// 2 * SPL_MAX_SPECIES doubles (min, max interleaved per species).
hipError_t launch_scalar_range(const ProjK &pk, int n_species, int log10, double *out_minmax,
                               hipStream_t s) {
  unsigned long long *mm = reinterpret_cast<unsigned long long *>(out_minmax);
  double *out = out_minmax + 2 * SPL_MAX_SPECIES;
  hipLaunchKernelGGL(k_init_minmax, dim3(1), dim3(64), 0, s, mm, n_species);
  if (pk.n > 0) {
    const int g = grid_for(pk.n, kBlock * 16, 4096);
    hipLaunchKernelGGL(k_scalar_range, dim3(g), dim3(kBlock), 0, s, pk, n_species, log10, mm);
  }
  hipLaunchKernelGGL(k_decode_minmax, dim3(1), dim3(64), 0, s, mm, n_species, out);
  return hipGetLastError();
}

}  // namespace spl
