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
// over the spans.  V views of the same particles (V = 2 for pairs of views of
// a batch): each particle's attributes are read once and projected for every
// view, each view with its own records, spans, totals and histogram (view v's
// bins numbered from A.hoff[v] on: 32-bit bins for one view, two 16-bit bins
// per LDS word for a pair).  Views of one launch share the particle arrays of
// A.P[0]; with V > 1 none is depth-sorted (no absorption is read).
template <int V>
struct ProjArgs {
  ProjK P[V];
  TileK tk[V];
  float4 *rec[V];
  float2 *rec2[V];
  uint2 *span[V];
  Totals *tot[V];
  uint32_t *counts[V];
  int hoff[V];
};

template <bool kCount, int kDt, int V>
__global__ __launch_bounds__(kBlock) void k_project(ProjArgs<V> A, int write_inactive) {
  extern __shared__ uint32_t hist[];
  __shared__ unsigned int s_act[V], s_large[V];
  // the species' looks, read per lane (the species select would otherwise
  // keep every look in scalar registers)
  __shared__ LookK s_looks[V][SPL_MAX_SPECIES];
  const ProjK &P0 = A.P[0];
  const int nh = A.hoff[V - 1] + A.tk[V - 1].n_tiles + A.tk[V - 1].n_ctiles;
  if (threadIdx.x < V) {
    s_act[threadIdx.x] = 0;
    s_large[threadIdx.x] = 0;
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (threadIdx.x < SPL_MAX_SPECIES) s_looks[v][threadIdx.x] = A.P[v].looks[threadIdx.x];
  const int nw = V == 1 ? nh : (nh + 1) / 2;  // histogram words
  if (kCount)
    for (int i = threadIdx.x; i < nw; i += kBlock) hist[i] = 0;
  __syncthreads();
  unsigned int my_act[V], my_large[V];
#pragma unroll
  for (int v = 0; v < V; ++v) my_act[v] = my_large[v] = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  // uniform trip count: the counting helpers need every lane of the wave
  for (int64_t kb = (int64_t)blockIdx.x * kBlock; kb < P0.n; kb += stride) {
    const int64_t k = kb + threadIdx.x;
    uint2 spn[V];
#pragma unroll
    for (int v = 0; v < V; ++v) spn[v] = make_uint2(kInactive, kInactive);
    if (k < P0.n) {
      const float x = P0.x[k], y = P0.y[k], z = P0.z[k];
      const float h = load_attr_t<kDt>(P0.h, k) * P0.h_scale;
      const float I = load_attr_t<kDt>(P0.inten, k) * P0.i_scale;
      const float s = load_attr_t<kDt>(P0.scal, k) * P0.s_scale;
      const int sp = P0.species ? (int)P0.species[k] : 0;
      const float a_in = (V == 1 && P0.mode == SPL_SORTED) ? P0.absorb[k] : 0.0f;
      // (one view at a time: unrolled, the views' live values would double
      // the registers and halve the waves per SIMD)
#pragma unroll 1
      for (int v = 0; v < V; ++v) {
        const ProjK &P = A.P[v];
        const TileK &tk = A.tk[v];
        const float a = (P.mode == SPL_SORTED) ? a_in : 0.0f;
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
        const LookK L = s_looks[v][in_ok ? sp : 0];
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
        uint2 sv = make_uint2(kInactive, kInactive);
        if (keep) sv = record_span(o0, o1.x, tk);
        const bool active = sv.x != kInactive;
        // (constant indices only: a run-time index would put the arrays in
        // scratch memory)
        if (v == 0)
          spn[0] = sv;
        else
          spn[V - 1] = sv;
        if (active) {
          const unsigned int lg = (sv.y & kLargeFlag) ? 1u : 0u;
          if (v == 0) {
            ++my_act[0];
            my_large[0] += lg;
          } else {
            ++my_act[V - 1];
            my_large[V - 1] += lg;
          }
        }
        if (active || write_inactive) {
          if (!active) {
            o0 = make_float4(0.f, 0.f, 0.f, 0.f);
            o1 = o0;
            o2 = make_float2(0.f, 0.f);
          }
          A.rec[v][2 * k] = o0;
          A.rec[v][2 * k + 1] = o1;
          if (A.rec2[v]) A.rec2[v][k] = o2;
        }
        A.span[v][k] = sv;
      }
    }
    // every lane of the wave takes part
    if (kCount) {
      if (V == 1) {
        count_span(spn[0], k, A.rec[0], A.tk[0], hist);
      } else {
        // two 16-bit bins per LDS word (the host launches pairs only when no
        // workgroup takes 2^16 particles, so no half carries into the other)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const uint32_t o = (uint32_t)A.hoff[v];
          count_span_with(spn[v], k, A.rec[v], A.tk[v], [&](uint32_t bin, uint32_t c) {
            const uint32_t b = o + bin;
            atomicAdd(&hist[b >> 1], c << ((b & 1u) * 16u));
          });
        }
      }
    }
  }
  if (kCount) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int nb = A.tk[v].n_tiles + A.tk[v].n_ctiles;
      for (int i = threadIdx.x; i < nb; i += kBlock) {
        uint32_t c;
        if (V == 1) {
          c = hist[i];
        } else {
          const uint32_t b = (uint32_t)A.hoff[v] + (uint32_t)i;
          c = (hist[b >> 1] >> ((b & 1u) * 16u)) & 0xffffu;
        }
        if (c) atomicAdd(&A.counts[v][i], c);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    if (my_act[v]) atomicAdd(&s_act[v], my_act[v]);
    if (my_large[v]) atomicAdd(&s_large[v], my_large[v]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      Totals *tot = A.tot[v];
      if (!tot) continue;
      if (s_act[v]) atomicAdd(&tot->n_active, (unsigned long long)s_act[v]);
      if (s_large[v]) atomicAdd(&tot->n_large, (unsigned long long)s_large[v]);
    }
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

template <int V>
static hipError_t launch_project_v(const ProjArgs<V> &A, int write_inactive, bool count,
                                   hipStream_t s) {
  const ProjK &pk = A.P[0];
  auto launch = [&](auto kernel, int g, size_t sh) {
    hipLaunchKernelGGL(kernel, dim3(g), dim3(kBlock), sh, s, A, write_inactive);
  };
  if (count) {
    // fewer, longer-lived workgroups: each flushes its histogram once
    const int g = grid_for(pk.n, kBlock, 4096);
    const int nh = A.hoff[V - 1] + A.tk[V - 1].n_tiles + A.tk[V - 1].n_ctiles;
    const size_t sh = (size_t)(V == 1 ? nh : (nh + 1) / 2) * sizeof(uint32_t);
    if (pk.dtype == SPL_BF16)
      launch(k_project<true, SPL_BF16, V>, g, sh);
    else if (pk.dtype == SPL_F16)
      launch(k_project<true, SPL_F16, V>, g, sh);
    else
      launch(k_project<true, SPL_F32, V>, g, sh);
  } else {
    const int g = grid_for(pk.n, kBlock, 8192);
    if (pk.dtype == SPL_BF16)
      launch(k_project<false, SPL_BF16, V>, g, 0);
    else if (pk.dtype == SPL_F16)
      launch(k_project<false, SPL_F16, V>, g, 0);
    else
      launch(k_project<false, SPL_F32, V>, g, 0);
  }
  return hipGetLastError();
}

hipError_t launch_project(const ProjK &pk, const TileK &tk, float *rec, float *rec2, uint2 *span,
                          int write_inactive, Totals *tot, hipStream_t s, uint32_t *counts) {
  if (pk.n == 0) return hipSuccess;
  ProjArgs<1> A;
  A.P[0] = pk;
  A.tk[0] = tk;
  A.rec[0] = reinterpret_cast<float4 *>(rec);
  A.rec2[0] = reinterpret_cast<float2 *>(rec2);
  A.span[0] = span;
  A.tot[0] = tot;
  A.counts[0] = counts;
  A.hoff[0] = 0;
  return launch_project_v(A, write_inactive, counts && project_counts(tk), s);
}

bool project_pair_ok(const ProjK &a, const TileK &ta, const ProjK &b, const TileK &tb) {
  // 16-bit bins: every workgroup of the counting grid takes < 2^16 particles
  const int64_t per_wg = (a.n + 4095) / 4096 + kBlock;
  return a.mode != SPL_SORTED && b.mode != SPL_SORTED && project_counts(ta) &&
         project_counts(tb) && a.n == b.n && a.x == b.x && a.dtype == b.dtype &&
         per_wg < 65536;
}

hipError_t launch_project_pair(const ProjK pk[2], const TileK tk[2], float *const rec[2],
                               uint2 *const span[2], Totals *const tot[2],
                               uint32_t *const counts[2], hipStream_t s) {
  if (pk[0].n == 0) return hipSuccess;
  if (!project_pair_ok(pk[0], tk[0], pk[1], tk[1])) return hipErrorInvalidValue;
  ProjArgs<2> A;
  for (int v = 0; v < 2; ++v) {
    A.P[v] = pk[v];
    A.tk[v] = tk[v];
    A.rec[v] = reinterpret_cast<float4 *>(rec[v]);
    A.rec2[v] = nullptr;
    A.span[v] = span[v];
    A.tot[v] = tot[v];
    A.counts[v] = counts[v];
  }
  A.hoff[0] = 0;
  A.hoff[1] = tk[0].n_tiles + tk[0].n_ctiles;
  return launch_project_v(A, 0, true, s);
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
