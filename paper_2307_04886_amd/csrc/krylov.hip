// Conjugate gradients in double on A x = b (level 0, colour-sorted
// numbering), preconditioned by the symmetric V-cycle in double or float
// (the method as the preconditioner of a Krylov solver, the extension named
// in the paper's conclusion, Sec. 6).  Flexible form with the Polak-Ribiere
// coefficient, which keeps the local A-orthogonality of successive directions when the preconditioner
// carries float rounding.  One iteration:
//   z = B r;  beta = (r.z - r_old.z) / rho;  rho = r.z;  p = z + beta p;
//   q = A p;  alpha = rho / p.q;  x += alpha p;  r_old = r;  r -= alpha q.
// Starting from p = 0, r_old = 0, rho = 1, the first iteration gives p = z.
// Every dot product is a fixed-grid partial sum plus a one-block tree sum
// (deterministic); the scalars stay on the device.
#include "rows.hpp"

namespace gmg {

namespace {

constexpr int kChunkSpmv = 8;

__global__ void k_kry_init(double* p, double* r_old, int64_t n, double* scal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    p[i] = 0.0;
    r_old[i] = 0.0;
  }
  if (i == 0) {
    scal[KS_RHO] = 1.0;
    scal[KS_BETA] = 0.0;
    scal[KS_ALPHA] = 0.0;
  }
}

// partials of r.z and r_old.z
template <class V>
__global__ void __launch_bounds__(kBlock) k_kry_dots(const double* __restrict__ r, const double* __restrict__ r_old,
                                                     const V* __restrict__ z, int64_t n, double* part) {
  double a = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double zi = (double)z[i];
    a += r[i] * zi;
    c += r_old[i] * zi;
  }
  a = block_sum(a);
  c = block_sum(c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[kNormBlocks + blockIdx.x] = c;
  }
}

__device__ inline double finish_sum(const double* part) {
  double s = 0.0;
  for (int i = threadIdx.x; i < kNormBlocks; i += kBlock) s += part[i];
  return block_sum(s);
}

__global__ void __launch_bounds__(kBlock) k_kry_beta(const double* part, double* scal) {
  const double rho_new = finish_sum(part);
  const double rz_old = finish_sum(part + kNormBlocks);
  if (threadIdx.x == 0) {
    scal[KS_BETA] = (rho_new - rz_old) / scal[KS_RHO];
    scal[KS_RHO] = rho_new;
  }
}

template <class V>
__global__ void k_kry_p(const V* __restrict__ z, const double* __restrict__ scal, double* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = scal[KS_BETA];
  p[i] = (double)z[i] + beta * p[i];
}

// q = A p, and partials of p.q
__global__ void __launch_bounds__(kBlock) k_kry_spmv(SellView A, const double* __restrict__ p, double* __restrict__ q,
                                                     int64_t n, double* part) {
  double s = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
    const double v = row_sum_seq<kChunkSpmv>(A, (int32_t)r, p, -1);
    q[r] = v;
    s += p[r] * v;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[2 * kNormBlocks + blockIdx.x] = s;
}

// alpha = rho / p.q; a non-positive curvature or rho means A (or B) is not SPD
__global__ void __launch_bounds__(kBlock) k_kry_alpha(const double* part, double* scal, int32_t* flags) {
  const double pq = finish_sum(part + 2 * kNormBlocks);
  if (threadIdx.x == 0) {
    const double rho = scal[KS_RHO];
    if (!(pq > 0.0) || !(rho > 0.0)) {
      atomicOr(flags, F_NOT_SPD);
      scal[KS_ALPHA] = 0.0;
    } else {
      scal[KS_ALPHA] = rho / pq;
    }
  }
}

// x += alpha p; r_old = r; r -= alpha q; partials of r.r
__global__ void __launch_bounds__(kBlock) k_kry_update(double* __restrict__ x, const double* __restrict__ p,
                                                       const double* __restrict__ q, double* __restrict__ r,
                                                       double* __restrict__ r_old, const double* __restrict__ scal,
                                                       int64_t n, double* part) {
  const double alpha = scal[KS_ALPHA];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    x[i] = x[i] + alpha * p[i];
    const double ri = r[i];
    r_old[i] = ri;
    const double rn = ri - alpha * q[i];
    r[i] = rn;
    s += rn * rn;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_kry_norm(const double* part, double* scal) {
  const double s = finish_sum(part);
  if (threadIdx.x == 0) scal[KS_NORM] = sqrt(s);
}

// out[e] = scale * u_i * v_col(e) for every entry e of row i: the gradient of a
// loss with respect to the stored entries of A (u = adjoint, v = solution).
__global__ void k_pattern_outer(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const double* __restrict__ u, const double* __restrict__ v, double scale,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ui = scale * u[i];
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) out[e] = ui * v[col[e]];
}

}  // namespace

void pattern_outer(int64_t n, const int32_t* rp, const int32_t* col, const double* u, const double* v,
                   double scale, double* out, hipStream_t s) {
  k_pattern_outer<<<blocks_for(n), kBlock, 0, s>>>(n, rp, col, u, v, scale, out);
}

void kry_init(Krylov& k, int64_t n, hipStream_t s) {
  k_kry_init<<<blocks_for(n), kBlock, 0, s>>>(k.p, k.r_old, n, k.scal);
}

template <class V>
void kry_direction(Krylov& k, const V* z, int64_t n, hipStream_t s) {
  k_kry_dots<V><<<kNormBlocks, kBlock, 0, s>>>(k.r, k.r_old, z, n, k.part);
  k_kry_beta<<<1, kBlock, 0, s>>>(k.part, k.scal);
  k_kry_p<V><<<blocks_for(n), kBlock, 0, s>>>(z, k.scal, k.p, n);
}

void kry_step(Krylov& k, const Level& l0, double* x, int32_t* flags, hipStream_t s) {
  const int64_t n = l0.n;
  k_kry_spmv<<<kNormBlocks, kBlock, 0, s>>>(l0.view.A, k.p, k.q, n, k.part);
  k_kry_alpha<<<1, kBlock, 0, s>>>(k.part, k.scal, flags);
  k_kry_update<<<kNormBlocks, kBlock, 0, s>>>(x, k.p, k.q, k.r, k.r_old, k.scal, n, k.part);
  k_kry_norm<<<1, kBlock, 0, s>>>(k.part, k.scal);
}

template void kry_direction<double>(Krylov&, const double*, int64_t, hipStream_t);
template void kry_direction<float>(Krylov&, const float*, int64_t, hipStream_t);

}  // namespace gmg
