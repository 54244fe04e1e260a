// Chinese remainder reconstruction of integer products from their residues
// (Section 5.2: the multimodular product recovered by the CRT, exact once the
// moduli's product M exceeds the entries, eq. CRT2).
//
// Per entry, on the device:
//   1. Garner's mixed-radix digits: X = v_0 + p_0 (v_1 + p_1 (v_2 + ...)),
//      0 <= v_j < p_j, with v_j = (r_j - X_{j-1}) (p_0 ... p_{j-1})^{-1} mod p_j
//      and X_{j-1} mod p_j evaluated by Horner over v_{j-1} ... v_0.  Every
//      step is binary64 modular arithmetic: Alg. 2 for the products, Alg. 1
//      for the reductions, all factors below the modulus and p <= 2^52 / 3
//      (Prop. Joris's range, x y <= 2^(t-1) p / 3).
//   2. The digits into 64-bit limbs by Horner from the top, acc = acc p_i +
//      v_i with 64 x 64 -> 128-bit limb products.
// The inverses (p_0 ... p_{j-1})^{-1} mod p_j and the limb count of M come
// from the host; p_i mod p_j is tabulated in LDS per workgroup.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

#include "mmp_internal.h"

namespace mmp {
namespace {

constexpr int kMaxModuli = 64;
constexpr uint64_t kRecPMax = (1ull << 52) / 3;  // Alg. 2 with both factors below p

struct RecArgs {
  const double* C[kMaxModuli];
  double p[kMaxModuli], q[kMaxModuli], inv[kMaxModuli];
  int act[kMaxModuli];  // limbs of p_i p_{i+1} ... p_{s-1}, for Horner step i
  int64_t ldc, m, n, ldo;
  uint64_t* out;
  int s, limbs;
};

// Alg. 1: x mod p for integer 0 <= x < 2^53.
__device__ __forceinline__ double rec_fmod(double x, double p, double q) {
  const double c = floor(x * q);
  double d = fma(-c, p, x);
  d = (d >= p) ? d - p : d;
  d = (d < 0.0) ? d + p : d;
  return d;
}

// Alg. 2: x y mod p for 0 <= x, y < p <= 2^52 / 3.
__device__ __forceinline__ double rec_mulmod(double x, double y, double p, double q) {
  const double h = x * y;
  const double l = fma(x, y, -h);
  const double c = floor(h * q);
  const double d = fma(-c, p, h);
  double e = d + l;
  e = (e >= p) ? e - p : e;
  e = (e < 0.0) ? e + p : e;
  return e;
}

// (t c + v) mod p for 0 <= t, c < p <= 2^52 / 3 and 0 <= v < 2^52: Alg. 2
// without its corrections leaves e = t c - b p in [-p, 2p), so
// e + v + p lies in [0, 2^53) and one Alg. 1 finishes.
__device__ __forceinline__ double rec_muladd(double t, double c, double v, double p, double q) {
  const double h = t * c;
  const double l = fma(t, c, -h);
  const double b = floor(h * q);
  const double d = fma(-b, p, h);
  const double e = d + l;
  return rec_fmod((e + p) + v, p, q);
}

// NT threads per workgroup; LDS holds the p_i mod p_j table and NT columns of
// s digits.
template <int LMAX, int NT>
__global__ __launch_bounds__(NT) void crt_reconstruct_kernel(const RecArgs a) {
  constexpr int kRecThreads = NT;
  extern __shared__ double lds[];
  const int s = a.s;
  double* pm = lds;                   // [s][s]: p_i mod p_j at i * s + j
  double* vcol = lds + s * s;         // [s][kRecThreads]: this thread's digits
  const int tid = threadIdx.x;
  for (int x = tid; x < s * s; x += kRecThreads) {
    const int i = x / s, j = x - i * s;
    pm[x] = rec_fmod(a.p[i], a.p[j], a.q[j]);
  }
  __syncthreads();
  const int64_t total = a.m * a.n;
  for (int64_t e = (int64_t)blockIdx.x * kRecThreads + tid; e < total; e += (int64_t)gridDim.x * kRecThreads) {
    const int64_t row = e / a.n, col = e - row * a.n;
    const int64_t off = row * a.ldc + col;
    // all residues first (independent loads), then Garner in place:
    // v_0 = r_0; v_j from r_j and X_{j-1} mod p_j
    for (int j = 0; j < s; j++) vcol[j * kRecThreads + tid] = a.C[j][off];
    for (int j = 1; j < s; j++) {
      const double pj = a.p[j], qj = a.q[j];
      double t = rec_fmod(vcol[(j - 1) * kRecThreads + tid], pj, qj);
      for (int i = j - 2; i >= 0; i--) t = rec_muladd(t, pm[i * s + j], vcol[i * kRecThreads + tid], pj, qj);
      double d = vcol[j * kRecThreads + tid] - t;
      d = (d < 0.0) ? d + pj : d;
      vcol[j * kRecThreads + tid] = rec_mulmod(d, a.inv[j], pj, qj);
    }
    // limbs: acc = v_{s-1}, then acc = acc p_i + v_i for i = s-2 .. 0
    uint64_t acc[LMAX];
#pragma unroll
    for (int w = 0; w < LMAX; w++) acc[w] = 0;
    acc[0] = (uint64_t)vcol[(s - 1) * kRecThreads + tid];
    for (int i = s - 2; i >= 0; i--) {
      const uint64_t pi = (uint64_t)a.p[i];
      uint64_t carry = (uint64_t)vcol[i * kRecThreads + tid];
      const int act = a.act[i];  // limbs that can be nonzero after this step
#pragma unroll
      for (int w = 0; w < LMAX; w++) {
        if (w < act) {
          const unsigned __int128 t = (unsigned __int128)acc[w] * pi + carry;
          acc[w] = (uint64_t)t;
          carry = (uint64_t)(t >> 64);
        }
      }
    }
#pragma unroll
    for (int w = 0; w < LMAX; w++)
      if (w < a.limbs) a.out[((int64_t)w * a.m + row) * a.ldo + col] = acc[w];
    for (int w = LMAX; w < a.limbs; w++) a.out[((int64_t)w * a.m + row) * a.ldo + col] = 0;
  }
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// x^{-1} mod p for gcd(x, p) = 1, 0 <= x < p (extended Euclid).
uint64_t inv_mod(uint64_t x, uint64_t p) {
  __int128 r0 = (__int128)p, r1 = (__int128)x, t0 = 0, t1 = 1;
  while (r1 != 0) {
    const __int128 qq = r0 / r1;
    __int128 tmp = r0 - qq * r1;
    r0 = r1;
    r1 = tmp;
    tmp = t0 - qq * t1;
    t0 = t1;
    t1 = tmp;
  }
  if (t0 < 0) t0 += p;
  return (uint64_t)t0;
}

// Number of 64-bit limbs of prod(p[lo..hi)).
int limbs_of_product(const uint64_t* p, int lo, int hi) {
  std::vector<uint64_t> x(1, 1);
  for (int i = lo; i < hi; i++) {
    unsigned __int128 carry = 0;
    for (auto& w : x) {
      const unsigned __int128 t = (unsigned __int128)w * p[i] + carry;
      w = (uint64_t)t;
      carry = t >> 64;
    }
    if (carry) x.push_back((uint64_t)carry);
  }
  int n = (int)x.size();
  while (n > 1 && x[n - 1] == 0) n--;
  return n;
}

// 128 threads up to 32 moduli (at most 40 KB of LDS), 64 beyond (at most 64 KB).
template <int LMAX>
int launch_rec(const RecArgs& a, void* stream) {
  const int64_t total = a.m * a.n;
  const int nt = a.s <= 32 ? 128 : 64;
  const int64_t blocks = std::min<int64_t>((total + nt - 1) / nt, 16384);
  const size_t shmem = sizeof(double) * ((size_t)a.s * a.s + (size_t)a.s * nt);
  if (nt == 128)
    hipLaunchKernelGGL((crt_reconstruct_kernel<LMAX, 128>), dim3((unsigned)blocks), dim3(128), shmem,
                       (hipStream_t)stream, a);
  else
    hipLaunchKernelGGL((crt_reconstruct_kernel<LMAX, 64>), dim3((unsigned)blocks), dim3(64), shmem,
                       (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace
}  // namespace mmp

using namespace mmp;

extern "C" int mmp_crt_reconstruct(const double* const* C, int64_t ldc, const uint64_t* moduli, int nmoduli,
                                   int64_t m, int64_t n, uint64_t* out, int64_t ldo, int limbs, void* stream) {
  try {
    if (m < 0 || n < 0 || nmoduli < 1 || nmoduli > kMaxModuli || !moduli || !C) return MMP_EINVAL;
    for (int i = 0; i < nmoduli; i++)
      if (moduli[i] < 2 || moduli[i] > kRecPMax) return MMP_EINVAL;
    for (int i = 0; i < nmoduli; i++)
      for (int j = i + 1; j < nmoduli; j++)
        if (gcd_u64(moduli[i], moduli[j]) != 1) return MMP_EINVAL;
    const int lm = limbs_of_product(moduli, 0, nmoduli);
    if (limbs < lm) return MMP_EINVAL;  // some X below M would not fit
    if (m == 0 || n == 0) return MMP_OK;
    if (!out || ldc < n || ldo < n) return MMP_EINVAL;
    for (int i = 0; i < nmoduli; i++) {
      if (!C[i]) return MMP_EINVAL;
      if (ranges_overlap(out, span_bytes((int64_t)limbs * m, n, ldo), C[i], span_bytes(m, n, ldc))) return MMP_EINVAL;
    }
    RecArgs a;
    std::memset(&a, 0, sizeof(a));
    a.s = nmoduli;
    a.limbs = limbs;
    a.ldc = ldc;
    a.m = m;
    a.n = n;
    a.ldo = ldo;
    a.out = out;
    for (int j = 0; j < nmoduli; j++) {
      a.C[j] = C[j];
      a.p[j] = (double)moduli[j];
      a.q[j] = 1.0 / (double)moduli[j];
      // (p_0 ... p_{j-1})^{-1} mod p_j
      unsigned __int128 prod = 1;
      for (int i = 0; i < j; i++) prod = (prod * (moduli[i] % moduli[j])) % moduli[j];
      a.inv[j] = j == 0 ? 0.0 : (double)inv_mod((uint64_t)prod, moduli[j]);
      a.act[j] = limbs_of_product(moduli, j, nmoduli);
    }
    int e;
    if (lm <= 2)
      e = launch_rec<2>(a, stream);
    else if (lm <= 4)
      e = launch_rec<4>(a, stream);
    else if (lm <= 8)
      e = launch_rec<8>(a, stream);
    else if (lm <= 16)
      e = launch_rec<16>(a, stream);
    else if (lm <= 28)
      e = launch_rec<28>(a, stream);
    else
      e = launch_rec<56>(a, stream);
    return hip_status(e);
  } catch (...) {
    return MMP_ENOMEM;
  }
}
