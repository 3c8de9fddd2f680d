// gf_monitor.hip -- the unitarity monitor: the largest deviation of U U^dag
// from the unit matrix over all links of a field, for gf_unitarity and the
// drivers' checks (GF_FLAG_MONITOR).
#include "gf_host.hpp"

namespace {

// largest |(A A^dag)_ab - delta_ab| of one link; NaN anywhere gives +Inf
__device__ __forceinline__ double link_unitarity(const Su3<double>& A) {
  double d = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      double re = 0, im = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // A_ak conj(A_bk)
        re += A.e[a][k].re * A.e[b][k].re + A.e[a][k].im * A.e[b][k].im;
        im += A.e[a][k].im * A.e[b][k].re - A.e[a][k].re * A.e[b][k].im;
      }
      if (a == b) re -= 1.0;
      const double m = sqrt(re * re + im * im);
      d = (m > d || m != m) ? m : d;
    }
  return d != d ? INFINITY : d;
}

// grid (ceil(vh / kBlock), 8): blockIdx.y = p*4 + mu; one partial per block
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_unitarity(const v2<T>* __restrict__ U, const uint32_t vh,
                                                      const uint32_t vp, double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
  double d = 0;
  if (h < vh) {
    Su3<double> A;
    load_link_f64<T, NC>(U + link_offset<NC>(vp, blockIdx.y >> 2, blockIdx.y & 3, h), A);
    d = link_unitarity(A);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = lds[0];
    for (int k = 1; k < kBlock / 64; ++k) m = fmax(m, lds[k]);
    partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = m;
  }
}

// one block: the largest of n partials into out[0]
__global__ __launch_bounds__(kBlock) void k_max_finish(const double* __restrict__ partial,
                                                       const uint32_t n, double* __restrict__ out) {
  __shared__ double lds[kBlock / 64];
  double d = 0;
  for (uint32_t i = threadIdx.x; i < n; i += kBlock) d = fmax(d, partial[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = lds[0];
    for (int k = 1; k < kBlock / 64; ++k) m = fmax(m, lds[k]);
    out[0] = m;
  }
}

}  // namespace

gf_status unitarity_launch(gf_ctx* c, const void* U, const gf_geom* g, double* out) {
  const Lat L = make_lat(g);
  const unsigned bx = blocks_for(L.vh);
  const size_t n = (size_t)bx * 8;
  gf_status st = ensure_partial(c, n);
  if (st != GF_OK) return st;
  with_type(g, [&]<typename T, int NC>() {
    hipLaunchKernelGGL((k_unitarity<T, NC>), dim3(bx, 8), dim3(kBlock), 0, c->stream,
                       (const v2<T>*)U, L.vh, L.vp, c->partial);
  });
  hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(kBlock), 0, c->stream, (const double*)c->partial,
                     (uint32_t)n, out);
  return launch_check(c, "gf_unitarity");
}

gf_status gf_unitarity(gf_ctx* c, const void* U, const gf_geom* g, double* dev_out) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_unitarity");
  if (!U || !dev_out) return fail(c, GF_ERR_ARG, "gf_unitarity: NULL pointer");
  return unitarity_launch(c, U, g, dev_out);
}
