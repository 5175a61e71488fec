// gfmc_kernels.hip -- gfx950 kernels of the GFMC hot path.
//
// Per proposal and chain (Algorithm 1, inner loop body; Section 2.2):
//   k_propose  : Philox draw of site and new direction, bond changes Delta_{n,o}
//   k_step     : one step of the three-term Chebyshev recursion (equation
//                "recursive") for the 7 start vectors, matrix-free, fused with
//                the Gram sums that give two moments per step (equation "mu2")
//   k_resident : the same recursion for small lattices, all steps of a
//                proposal in one LDS-resident workgroup per chain
//   k_moments  : deferred, compensated sum of the per-block Gram partials and
//                assembly of mu_n^{jk}, n < M
//   k_recon    : contraction to the 2x2 block, damping kernel, node transform
//                by radix-2 FFT (equations "green_short", "green_fft",
//                "mu_to_mu_tilde"), determinant (equation "d_z_green"),
//                continuous phase, energy integral (equation "d_seff2"),
//                Metropolis test and spin update
//   k_magnetization: |sum_i S_i| / N at the end of a sweep
#include <type_traits>

#include "gfmc_device.h"

namespace gfmc {

typedef double d4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ Philox ------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter (c0, c1, 0, 0).
__device__ inline void philox(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1,
                              uint64_t out[4]) {
  uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B97F4A7C15ULL;
      k1 += 0xBB67AE8584CAA73BULL;
    }
    const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
    uint64_t hi0 = __umul64hi(m0, x0), lo0 = m0 * x0;
    uint64_t hi1 = __umul64hi(m1, x2), lo1 = m1 * x2;
    uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// Global address space: loads and stores through such pointers are global,
// not flat, instructions (a flat access also counts against the LDS wait
// counter).
#define GLOBAL __attribute__((address_space(1)))

__device__ inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

__device__ inline void site_xyz(int i, int L, int& x, int& y, int& z) {
  x = i % L;
  y = (i / L) % L;
  z = i / (L * L);
}

__device__ inline int neighbor_site(int i, int d, int L) {
  int x, y, z;
  site_xyz(i, L, x, y, z);
  switch (d) {
    case 0: x = (x + 1 == L) ? 0 : x + 1; break;
    case 1: x = (x == 0) ? L - 1 : x - 1; break;
    case 2: y = (y + 1 == L) ? 0 : y + 1; break;
    case 3: y = (y == 0) ? L - 1 : y - 1; break;
    case 4: z = (z + 1 == L) ? 0 : z + 1; break;
    default: z = (z == 0) ? L - 1 : z - 1; break;
  }
  return x + L * (y + L * z);
}

// Half-row index of the neighbour of (x,y,z) in direction d.
__device__ inline int nb_half(int x, int y, int z, int d, int L) {
  switch (d) {
    case 0: x = (x + 1 == L) ? 0 : x + 1; break;
    case 1: x = (x == 0) ? L - 1 : x - 1; break;
    case 2: y = (y + 1 == L) ? 0 : y + 1; break;
    case 3: y = (y == 0) ? L - 1 : y - 1; break;
    case 4: z = (z + 1 == L) ? 0 : z + 1; break;
    default: z = (z == 0) ? L - 1 : z - 1; break;
  }
  return half_index(x, y, z, L);
}

__device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
  const uint32_t q = __umulhi(n, f.m);
  return q + ((q + 1u) * f.d <= n ? 1u : 0u);
}

// Row coordinates of half-row index h: h = k + (L/2)(y + L z).
__device__ inline void split_half(int h, const Desc& D, int& k, int& y, int& z) {
  const int r = (int)fdiv((uint32_t)h, D.div_hx);
  k = h - r * (D.L >> 1);
  z = (int)fdiv((uint32_t)r, D.div_L);
  y = r - z * D.L;
}

// Half-row indices of the six neighbours (the order of nb_half: x+1, x-1,
// y+1, y-1, z+1, z-1) of the site with half-row index h, row coordinates
// (k, y, z) and x = 2k + xb, by offsets from h: an x neighbour shares h or
// is the next or previous entry of the row (wrapping within it), the y and z
// neighbours are a row or a plane away (wrapping across the lattice).
__device__ inline void nb6_half(int h, int k, int xb, int y, int z, int L, int nh[6]) {
  const int hx = L >> 1, plane = hx * L, row = h - k;
  nh[0] = xb ? ((k + 1 == hx) ? row : h + 1) : h;
  nh[1] = xb ? h : ((k == 0) ? row + hx - 1 : h - 1);
  nh[2] = (y + 1 == L) ? h - hx * (L - 1) : h + hx;
  nh[3] = (y == 0) ? h + hx * (L - 1) : h - hx;
  nh[4] = (z + 1 == L) ? h - plane * (L - 1) : h + plane;
  nh[5] = (z == 0) ? h + plane * (L - 1) : h - plane;
}

// Hopping amplitude from the angles (equation "ht"), FP64.
__device__ inline void hop_angles(double ti, double pi_, double tj, double pj, double& re,
                                  double& im) {
  re = cos(0.5 * (ti - tj)) * cos(0.5 * (pi_ - pj));
  im = cos(0.5 * (ti + tj)) * sin(0.5 * (pi_ - pj));
}

template <typename T>
__device__ inline spn<T> make_spinor(double th, double ph) {
  double st, ct, sp, cp;
  sincos(0.5 * th, &st, &ct);
  sincos(0.5 * ph, &sp, &cp);
  spn<T> s;
  s.ar = (T)(ct * cp);
  s.ai = (T)(-ct * sp);
  s.br = (T)(st * cp);
  s.bi = (T)(st * sp);
  return s;
}

// sc <chi_i|chi_j> = sc t_ij with sc = -t/a: the element of the rescaled
// Hamiltonian Ht (t_ij as in equation "ht", from the cached half-angle
// factors), each element rounded once to the recursion precision T.
// In the FP32 recursion two roundings of the Hamiltonian dominate the error
// of the moments, not the rounding of the vectors: a scale -2t/a rounded to
// FP32 once multiplies every step's Ht by the same (1 + 4e-8), an error that
// grows coherently with the moment order, and amplitudes summed in FP32
// carry a few 1e-8 absolute error each.  Scaling each element by sc, not
// the step's sum by 2 sc (the steps then double exactly), and carrying sc
// as an FP32 pair hi + lo (so that its rounding acts on no element) removes
// the coherent part.  FP32 forms t_ij in FP32 arithmetic and the scaled
// element as fma(t, hi, t lo), keeping Ht exactly Hermitian; a float model
// of the recursion puts its moment error within 15 % of forming sc t_ij in
// FP64 and rounding once (whose FP64 products and conversions made the step
// kernels' arithmetic their bound in the pair form); FP64 forms it directly.
template <typename T>
__device__ inline void hop_spinor(const spn<T>& a, const spn<T>& b, const double sc, T& re,
                                  T& im) {
  const double ar = a.ar, ai = a.ai, br = a.br, bi = a.bi;
  const double cr = b.ar, ci = b.ai, dr = b.br, di = b.bi;
  re = (T)(sc * (ar * cr + ai * ci + br * dr + bi * di));
  im = (T)(sc * (ar * ci - ai * cr + br * di - bi * dr));
}
template <>
__device__ inline void hop_spinor<float>(const spn<float>& a, const spn<float>& b,
                                         const double sc, float& re, float& im) {
  // Ht stays Hermitian bit for bit: the element for (j, i) must be the exact
  // conjugate of the one for (i, j).  The real part's fused chain takes the
  // same products in the same order either way; the imaginary part is formed
  // from rounded products and their differences (no fusion), which only
  // change sign when i and j swap.
#pragma clang fp contract(off)
  const float sh = (float)sc, sl = (float)(sc - (double)sh);   // kernel-invariant
  float tr = a.bi * b.bi;
  tr = fmaf(a.br, b.br, tr);
  tr = fmaf(a.ai, b.ai, tr);
  tr = fmaf(a.ar, b.ar, tr);
  const float d1 = a.ar * b.ai - a.ai * b.ar;
  const float d2 = a.br * b.bi - a.bi * b.br;
  const float ti = d1 + d2;
  re = fmaf(tr, sh, tr * sl);
  im = fmaf(ti, sh, ti * sl);
}

// Per-field selects (a struct-valued ?: can go through scratch memory).
template <typename T>
__device__ inline spn<T> pick(bool c, const spn<T>& a, const spn<T>& b) {
  return spn<T>{c ? a.ar : b.ar, c ? a.ai : b.ai, c ? a.br : b.br, c ? a.bi : b.bi};
}
template <typename T>
__device__ inline cpx<T> pick(bool c, const cpx<T>& a, const cpx<T>& b) {
  return cpx<T>{c ? a.x : b.x, c ? a.y : b.y};
}

// (ar, ai) += (hr + i hi) a with the four products fused in a fixed order, so
// that every form of the step (one step or two per launch, the LDS-resident
// and the persistent kernels, whatever the compiler makes of the code around
// it) forms every vector value bit for bit alike.
template <typename T>
__device__ inline void cmac(T hr, T hi, const cpx<T>& a, T& ar, T& ai) {
  ar = fma(hr, a.x, ar);
  ar = fma(-hi, a.y, ar);
  ai = fma(hr, a.y, ai);
  ai = fma(hi, a.x, ai);
}

// Block b of a grid of nb blocks runs on XCD b % 8; give each XCD a
// contiguous range of logical blocks so that lattice planes that neighbour in
// z are processed under the same L2.
__device__ inline int xcd_remap(int b, int nb) {
  const int x = b & 7, i = b >> 3;
  const int base = nb >> 3, rem = nb & 7;
  return x * base + (x < rem ? x : rem) + i;
}

// -------------------------------------------------------------- propose ---
// One wave per chain: lane 0 draws the proposal (the FP64 trigonometry of a
// new direction), then lanes 0..5 each form the bond change to one neighbour,
// so the twelve hopping evaluations run side by side.
__global__ __launch_bounds__(64) void k_propose(const Desc* __restrict__ descs, int n) {
  // no FMA contraction: an unchanged spin must give Delta_{n,o} = 0 exactly
#pragma clang fp contract(off)
  const int c = blockIdx.x, lane = threadIdx.x;
  if (c >= n) return;
  const Desc& D = descs[c];
  Ctl* ctl = D.ctl;
  const GLOBAL double* th = (const GLOBAL double*)D.theta;
  const GLOBAL double* ph = (const GLOBAL double*)D.phi;
  const int mode = ctl->mode;
  const int L = D.L;
  int o = 0;
  double tn = 0.0, pn = 0.0, to = 0.0, po = 0.0;
  if (lane < 4) ctl->bar[lane] = 0u;
  if (lane == 0) {
    double u = 0.0, ua = 0.0, ub = 0.0;
    if (mode == 0) {
      uint64_t r[4];
      philox((uint64_t)ctl->index, 1ULL, D.seed, D.chain_id, r);
      o = (int)__umul64hi(r[0], (uint64_t)D.N);
      ua = u01(r[1]);
      ub = u01(r[2]);
      u = u01(r[3]);
    } else {
      o = ctl->site;
      tn = ctl->th_new;
      pn = ctl->ph_new;
    }
    to = th[o];
    po = ph[o];
    if (mode == 0) {
      if (D.proposal == GFMC_PROPOSE_CONE) {
        const double st = sin(to), ct = cos(to), sp = sin(po), cp = cos(po);
        const double S[3] = {st * cp, st * sp, ct};
        const double e1[3] = {ct * cp, ct * sp, -st};
        const double e2[3] = {-sp, cp, 0.0};
        const double ca = 1.0 - (1.0 - cos(D.cone)) * ua;
        const double sa = sqrt(fmax(0.0, (1.0 - ca) * (1.0 + ca)));
        const double psi = 2.0 * M_PI * ub;
        const double cs = cos(psi), ss = sin(psi);
        double Sn[3];
        for (int q = 0; q < 3; ++q) Sn[q] = ca * S[q] + sa * (cs * e1[q] + ss * e2[q]);
        tn = atan2(sqrt(Sn[0] * Sn[0] + Sn[1] * Sn[1]), Sn[2]);
        pn = atan2(Sn[1], Sn[0]);
        if (pn < 0) pn += 2.0 * M_PI;
      } else {
        tn = acos(1.0 - 2.0 * ua);
        pn = 2.0 * M_PI * ub;
      }
    }
    int x, y, z;
    site_xyz(o, L, x, y, z);
    ctl->parity_o = (x + y + z) & 1;
    ctl->o_half = half_index(x, y, z, L);
    ctl->start_site[0] = o;
    ctl->start_half[0] = half_index(x, y, z, L);
    ctl->th_old = to;
    ctl->ph_old = po;
    if (mode == 0) {
      ctl->site = o;
      ctl->th_new = tn;
      ctl->ph_new = pn;
      ctl->u = u;
    }
  }
  o = __shfl(o, 0);
  tn = __shfl(tn, 0);
  pn = __shfl(pn, 0);
  to = __shfl(to, 0);
  po = __shfl(po, 0);
  if (lane < 6) {
    const int d = lane, nb = neighbor_site(o, d, L);
    const double tj = th[nb], pj = ph[nb];
    int a, b, cc;
    site_xyz(nb, L, a, b, cc);
    ctl->start_site[1 + d] = nb;
    ctl->start_half[1 + d] = half_index(a, b, cc, L);
    // Delta_{n,o} = H'_{n,o} - H_{n,o} = -t (t'_{n o} - t_{n o})
    double r1, i1, r0, i0;
    hop_angles(tj, pj, tn, pn, r1, i1);
    hop_angles(tj, pj, to, po, r0, i0);
    ctl->delta[2 * d] = -D.t * (r1 - r0);
    ctl->delta[2 * d + 1] = -D.t * (i1 - i0);
  }
}

// ------------------------------------------------------------ Chebyshev ---

// Six neighbour-vector values of one site, stored contiguously.
template <typename T>
struct alignas(16) six {
  cpx<T> v[6];
};

// Loads and stores through global-address-space pointers as plain vector
// accesses (16-byte where the layout allows).
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ inline spn<float> ld(const GLOBAL spn<float>* p) {
  const f4v v = *(const GLOBAL f4v*)p;
  return {v.x, v.y, v.z, v.w};
}
__device__ inline spn<double> ld(const GLOBAL spn<double>* p) {
  const GLOBAL d2v* q = (const GLOBAL d2v*)p;
  const d2v a = q[0], b = q[1];
  return {a.x, a.y, b.x, b.y};
}
__device__ inline cpx<float> ld(const GLOBAL cpx<float>* p) {
  const f2v v = *(const GLOBAL f2v*)p;
  return {v.x, v.y};
}
__device__ inline cpx<double> ld(const GLOBAL cpx<double>* p) {
  const d2v v = *(const GLOBAL d2v*)p;
  return {v.x, v.y};
}
__device__ inline void st(GLOBAL cpx<float>* p, const cpx<float>& c) {
  f2v v = {c.x, c.y};
  *(GLOBAL f2v*)p = v;
}
__device__ inline void st(GLOBAL cpx<double>* p, const cpx<double>& c) {
  d2v v = {c.x, c.y};
  *(GLOBAL d2v*)p = v;
}
// Non-temporal forms: a thread's own a_{s-2} is read once and then
// overwritten, and a_s is read again only in later steps.
__device__ inline cpx<float> ld_nt(const GLOBAL cpx<float>* p) {
  const f2v v = __builtin_nontemporal_load((const GLOBAL f2v*)p);
  return {v.x, v.y};
}
__device__ inline cpx<double> ld_nt(const GLOBAL cpx<double>* p) {
  const d2v v = __builtin_nontemporal_load((const GLOBAL d2v*)p);
  return {v.x, v.y};
}
__device__ inline void st_nt(GLOBAL cpx<float>* p, const cpx<float>& c) {
  f2v v = {c.x, c.y};
  __builtin_nontemporal_store(v, (GLOBAL f2v*)p);
}
__device__ inline void st_nt(GLOBAL cpx<double>* p, const cpx<double>& c) {
  d2v v = {c.x, c.y};
  __builtin_nontemporal_store(v, (GLOBAL d2v*)p);
}
// Device-coherent forms for the persistent kernel: relaxed device-scope
// atomic loads of 8-byte words, which skip this compute unit's L1 and are
// served by the L2, so values other blocks stored in the previous step are
// read without invalidating any cache.
__device__ inline uint64_t ld_dev8(const GLOBAL void* p) {
  return __hip_atomic_load((const GLOBAL uint64_t*)p, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline cpx<float> ld_coh(const GLOBAL cpx<float>* p) {
  const f2v v = __builtin_bit_cast(f2v, ld_dev8(p));
  return {v.x, v.y};
}
__device__ inline cpx<double> ld_coh(const GLOBAL cpx<double>* p) {
  const GLOBAL uint64_t* q = (const GLOBAL uint64_t*)p;
  return {__builtin_bit_cast(double, ld_dev8(q)), __builtin_bit_cast(double, ld_dev8(q + 1))};
}

// Global storage of six values per site (the n-slots, the stored hopping
// rows): planes of 16-byte items, item i of plane q at q * stride + i, so a
// wave's access to one plane is one contiguous run (a 48- or 96-byte record
// per lane would spread each 16-byte access over three or six times as many
// cache lines).  FP32: 3 planes, complex values 2q and 2q + 1 in plane q;
// FP64: 6 planes, value q in plane q.  stride = items per plane (>= 2 half).
template <typename T>
struct Planes;
template <>
struct Planes<float> {
  GLOBAL f4v* p;
  size_t stride;
  __device__ six<float> ld(size_t i) const {
    six<float> r;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const f4v v = p[q * stride + i];
      r.v[2 * q] = {v.x, v.y};
      r.v[2 * q + 1] = {v.z, v.w};
    }
    return r;
  }
  __device__ void st(size_t i, const six<float>& r) const {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      f4v v = {r.v[2 * q].x, r.v[2 * q].y, r.v[2 * q + 1].x, r.v[2 * q + 1].y};
      p[q * stride + i] = v;
    }
  }
  __device__ six<float> ld_coh(size_t i) const {
    six<float> r;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const GLOBAL uint64_t* w = (const GLOBAL uint64_t*)(p + q * stride + i);
      const f2v a = __builtin_bit_cast(f2v, ld_dev8(w));
      const f2v b = __builtin_bit_cast(f2v, ld_dev8(w + 1));
      r.v[2 * q] = {a.x, a.y};
      r.v[2 * q + 1] = {b.x, b.y};
    }
    return r;
  }
  __device__ six<float> ld_nt(size_t i) const {
    six<float> r;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const f4v v = __builtin_nontemporal_load(p + q * stride + i);
      r.v[2 * q] = {v.x, v.y};
      r.v[2 * q + 1] = {v.z, v.w};
    }
    return r;
  }
  __device__ void st_nt(size_t i, const six<float>& r) const {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      f4v v = {r.v[2 * q].x, r.v[2 * q].y, r.v[2 * q + 1].x, r.v[2 * q + 1].y};
      __builtin_nontemporal_store(v, p + q * stride + i);
    }
  }
};
template <>
struct Planes<double> {
  GLOBAL d2v* p;
  size_t stride;
  __device__ six<double> ld(size_t i) const {
    six<double> r;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const d2v v = p[q * stride + i];
      r.v[q] = {v.x, v.y};
    }
    return r;
  }
  __device__ void st(size_t i, const six<double>& r) const {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      d2v v = {r.v[q].x, r.v[q].y};
      p[q * stride + i] = v;
    }
  }
  __device__ six<double> ld_coh(size_t i) const {
    six<double> r;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const GLOBAL uint64_t* w = (const GLOBAL uint64_t*)(p + q * stride + i);
      r.v[q] = {__builtin_bit_cast(double, ld_dev8(w)), __builtin_bit_cast(double, ld_dev8(w + 1))};
    }
    return r;
  }
  __device__ six<double> ld_nt(size_t i) const {
    six<double> r;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const d2v v = __builtin_nontemporal_load(p + q * stride + i);
      r.v[q] = {v.x, v.y};
    }
    return r;
  }
  __device__ void st_nt(size_t i, const six<double>& r) const {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      d2v v = {r.v[q].x, r.v[q].y};
      __builtin_nontemporal_store(v, p + q * stride + i);
    }
  }
};
template <typename T>
__device__ inline Planes<T> planes(void* base, size_t stride) {
  using I = typename std::conditional<sizeof(T) == 4, f4v, d2v>::type;
  return Planes<T>{(GLOBAL I*)base, stride};
}

// One step s >= 1 of the recursion (equation "recursive"), |a_1> = Ht|a_0>
// and |a_s> = 2 Ht|a_{s-1}> - |a_{s-2}> for s >= 2, for the 7 start vectors
// of every chain in the launch, with the elements of Ht = -(t/a) t_ij formed
// per bond in FP64 and rounded once (the factor 2 is exact).  The lattice is bipartite and Ht connects only opposite
// parities, so a^o_s lives on parity p(o)^(s&1) and the six neighbour
// vectors a^n_s on the other parity; each site therefore stores one value of
// a^o (o-slot) and six of a^n (n-slots) and a_{s+1} overwrites a_{s-1} in
// place.  Each thread owns PPT half-row indices; for each, the two sites of
// that index (one per parity): on one it forms a^o_s from the 6 neighbours,
// on the other the six a^n_s.
//
// Moments (equation "mu2", doubling): per step the kernel accumulates
//   P^{oo}_s = <a^o_s|a^o_s>, P^{de}_s = <a^{n_d}_s|a^{n_e}_s>,
//   Q^{oe}_s = <a^o_{s-1}|a^{n_e}_s>
// (the other pairs vanish on a bipartite lattice) as the 16x16 real Gram
// matrix of the per-site-pair vector
//   x = (Re/Im a^{n_0..5}_s, Re/Im a^o_{s-1}  at the n-site,  Re/Im a^o_s at the o-site)
// summed over the block on the FP64 matrix core, and stores the 49 real
// combinations per block (no reduction on the per-step critical path).
// The 49 real block sums from the per-wave 16x16 Gram matrices in gsum:
// t = 0: P^{oo}; 1..36: P^{de} (d <= e; diagonal -> Re, off-diagonal -> Re, Im);
// 37..48: Q^{oe} (Re, Im).
// Sum t of the 49 as G(p1) + sg G(p2) over entries p = 16 i + j of the Gram
// matrix, sg = +1 or -1, G(p) = sum of the four waves' entries p.
struct Combo {
  int p1, p2;
  double sg;
};
__device__ inline Combo gram_combo_index(int t) {
  if (t == 0) return {14 * 16 + 14, 15 * 16 + 15, 1.0};
  if (t < 37) {
    // P^{de}, d <= e: group d holds 1 + 2 (5 - d) sums (diagonal, then Re
    // and Im per e > d); found by an unrolled scan, not a loop
    const int idx0 = t - 1;
    int d = 0, base = 0;
#pragma unroll
    for (int q = 1; q <= 5; ++q) {
      const int cum = 12 * q - q * q;   // sums in groups 0 .. q-1
      if (idx0 >= cum) {
        base = cum;
        d = q;
      }
    }
    const int idx = idx0 - base;
    if (idx == 0) return {(2 * d) * 16 + 2 * d, (2 * d + 1) * 16 + 2 * d + 1, 1.0};
    const int e = d + 1 + (idx - 1) / 2;
    return ((idx - 1) & 1) ? Combo{(2 * d) * 16 + 2 * e + 1, (2 * d + 1) * 16 + 2 * e, -1.0}
                           : Combo{(2 * d) * 16 + 2 * e, (2 * d + 1) * 16 + 2 * e + 1, 1.0};
  }
  const int q = t - 37, e = q >> 1;
  return (q & 1) ? Combo{12 * 16 + 2 * e + 1, 13 * 16 + 2 * e, -1.0}
                 : Combo{12 * 16 + 2 * e, 13 * 16 + 2 * e + 1, 1.0};
}
// Sum over the NW waves' Gram matrices (in wave order) of the entries of one
// of the 49 sums.
template <int NW = 4>
__device__ inline double gram_combo(const double (*gsum)[256], const Combo& k) {
  double a = gsum[0][k.p1], b = gsum[0][k.p2];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    a += gsum[w][k.p1];
    b += gsum[w][k.p2];
  }
  return a + k.sg * b;
}

// Step index of a chain in a launch.  Lock-step launches (act_end == NULL)
// give every chain the launch's step s.  Round launches (act_end != NULL)
// pass the round r of a window in which each chain runs its proposals back
// to back, S steps each: the chain is at step (r - 1) mod S + 1 of its
// current proposal while r <= act_end[c] (its last active round), and idle
// after it; step 1 of each proposal runs in a launch of its own (it also
// writes the start vectors), so round launches skip it.  Returns 0 for a
// chain that does not step in this launch.
__device__ inline int chain_step(int s, const int* __restrict__ act_end, int c, int S) {
  if (!act_end) return s;
  if (s > act_end[c]) return 0;
  const int sl = (s - 1) % S + 1;
  return sl == 1 ? 0 : sl;
}

// Step s of the chain D on its logical block lb (BT threads, PPT
// half-row indices per thread): the stencil, the in-place update and the
// block's 49 Gram sums.  Shared by the one-launch-per-step kernel and the
// persistent single-chain kernel.
// The point after which all loads of a batch (one site, or a group of its
// directions) must have been issued.
#define STEP_LOADS_ISSUED() __builtin_amdgcn_sched_barrier(0)

// Hook between a step's vector updates and its Gram sums (the persistent
// kernel counts in at its step barrier there, so that the barrier's wait
// overlaps the sums); the one-step kernels pass this no-op.
struct NoArrive {
  __device__ void operator()() const {}
};

// The block's 49 Gram sums of step s from the 16 values of each thread's
// site pair, left in LDS by step s (xw[wave][lane][component]): the same
// v_mfma_f64_16x16x4 products, in the same order, as the staged form at the
// end of step_block, so both give the same partial sums bit for bit.  Every
// thread of the block must call it (it holds a block barrier).
template <int NW>
__device__ __forceinline__ void gram_rows(const Desc& D, const int lb, const int s,
                                          double (*xw)[64][17], double (*gsum)[256]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const double val = xw[w][16 * rr + 4 * m + (lane >> 4)][lane & 15];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(val, val, acc, 0, 0, 0);
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) gsum[w][(4 * r + (lane >> 4)) * 16 + (lane & 15)] = acc[r];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kNP)
    D.part[((size_t)(s - 1) * kNP + t) * D.nblk + lb] = gram_combo<NW>(gsum, gram_combo_index(t));
}

// The block's 49 Gram sums of step s from the 16 values of each thread's PPT
// site pairs (the column form below; step_block forms the same sums inline):
// v_mfma_f64_16x16x4 with A = B = 4 columns (site pairs) of 16
// components on the FP64 matrix core; each wave stages 16 site pairs at a
// time in LDS (4 rounds per pair slot), slot by slot.  Every thread of the
// block must call it (it holds a block barrier).
template <int PPT, int NW>
__device__ __forceinline__ void gram_staged(const Desc& D, const int lb, const int s,
                                            const double (&x)[PPT][16], double (*xs)[16][17],
                                            double (*gsum)[256]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      if ((lane >> 4) == rr) {
#pragma unroll
        for (int i = 0; i < 16; ++i) xs[w][lane & 15][i] = x[p][i];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double val = xs[w][4 * m + (lane >> 4)][lane & 15];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(val, val, acc, 0, 0, 0);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // result layout of v_mfma_f64_16x16x4: lane l, register r holds entry
  // (4r + l/16, l%16) of the 16x16 product
#pragma unroll
  for (int r = 0; r < 4; ++r) gsum[w][(4 * r + (lane >> 4)) * 16 + (lane & 15)] = acc[r];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kNP)
    D.part[((size_t)(s - 1) * kNP + t) * D.nblk + lb] = gram_combo<NW>(gsum, gram_combo_index(t));
}

template <typename T, bool FIRST, int PPT, bool HOPS, bool NT, bool COH = false,
          typename Arrive = NoArrive, int BT = kStepThreads>
__device__ __forceinline__ void step_block(const Desc& D, const int lb, const int s,
                                           double (*xs)[16][17], double (*gsum)[256],
                                           const Arrive& arrive = Arrive(),
                                           const cpx<T> (*hp)[6] = nullptr,
                                           double (*xw)[64][17] = nullptr) {
  const int L = D.L, half = D.half;
  const Ctl* ctl = D.ctl;
  const int pO = ctl->parity_o;
  const int po = pO ^ (s & 1);          // parity of the sites that carry a^o_s
  const int pn = po ^ 1;                // parity of the sites that carry a^n_s
  const int o_half = ctl->o_half;
  int sh[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) sh[e] = FIRST ? ctl->start_half[1 + e] : 0;
  const double hsc = -D.t / D.a;        // Ht = -(t/a) t_ij
  const T two = FIRST ? (T)1 : (T)2;     // |a_1> = Ht|a_0>, then 2 Ht|a_{s-1}> - |a_{s-2}>
  const GLOBAL spn<T>* sp = (const GLOBAL spn<T>*)D.spin;            // [2][half]
  GLOBAL cpx<T>* vo = (GLOBAL cpx<T>*)D.vec;                         // o-slots [2][half]
  const Planes<T> vn = planes<T>((cpx<T>*)D.vec + D.N, D.N);        // n-slots [2][half]
  const GLOBAL spn<T>* sp_o = sp + (size_t)po * half;
  const GLOBAL spn<T>* sp_n = sp + (size_t)pn * half;
  // stored hopping rows t_{i, n_d(i)} (HOPS): six<T>[2][half]
  const Planes<T> hrow = planes<T>(D.hop, D.N);

  // COH (persistent kernel): a neighbour value stored in the previous step by
  // another block, that is on another compute unit, is read past this
  // unit's L1; one this block stored went through the same L1 and loads as
  // usual (each block keeps its site pairs from step to step).  Its threads
  // also keep their site pair's twelve hopping amplitudes in registers for
  // the whole proposal (hp[q][d]: the site of parity q to its neighbour d,
  // formed by the same hop_spinor), so its steps load no spinors.
  //   It forms a step's Gram sums during the next step, while that step's
  // loads are in flight (gram_rows, from the 16 values per thread it leaves
  // in LDS): every thread of its blocks runs each step, a thread past the
  // lattice on the last site pair with its stores and values dropped, so
  // that the block barrier inside the sums is reached by all.
  constexpr int NW = BT / 64;   // waves per block
  auto nb_elsewhere = [&](int nhh) { return nhh / (BT * PPT) != lb; };
  double x[PPT][16];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
#pragma unroll
    for (int i = 0; i < 16; ++i) x[p][i] = 0.0;
    const int h0 = (lb * PPT + p) * BT + (int)threadIdx.x;
    const bool valid = h0 < half;
    if (!COH && !valid) continue;
    const int h = valid ? h0 : half - 1;
    int k, y, z;
    split_half(h, D, k, y, z);
    const int bo = (y + z + po) & 1, bn = bo ^ 1;   // x = 2k + b of the o- and n-site
    // a^o_s on the o-site.  Every load of the site is issued before its
    // arithmetic (one memory round trip): left to itself the compiler keeps
    // registers low by waiting for each direction's loads in turn, and the
    // kernel becomes bound by the latency of those round trips.
    //   One x neighbour of either site is the pair's other site (same
    // half-row index, other parity): the o-site takes that neighbour's
    // spinor and a^o_{s-1} from the n-site's own loads, the n-site takes the
    // o-site's spinor (three loads fewer per pair; the sums keep their order).
    // FP32 steps only: in FP64 the values held from one phase to the next
    // cost more registers than the three loads save (measured slower).
    constexpr bool DEDUP = sizeof(T) == 4;
    spn<T> s_o, s_n;   // the pair's own spinors
    cpx<T> aop;        // a^o_{s-1} at the n-site
    // The persistent kernel (one wave per SIMD, registers to spare) issues the
    // n-site's loads with the o-site's in FP32: one memory round trip per
    // step (16^3: 514 against 505 proposals/s; in FP64 the values overflow
    // into the accumulation registers and it measured 4 % slower).
    constexpr bool MERGE = COH && sizeof(T) == 4;
    six<T> anm[6], prevm;   // the n-site's neighbour and own values (MERGE)
    int nhn[6];   // the n-site's neighbours
    if (MERGE) nb6_half(h, k, bn, y, z, L, nhn);
    {
      int nh[6];
      nb6_half(h, k, bo, y, z, L, nh);
      const int dx = bo ? 0 : 1;   // the x direction whose neighbour is another pair
      spn<T> sj[6];
      six<T> row;
      cpx<T> an[6], pr = {(T)0, (T)0};
      if (HOPS) {
        row = hrow.ld((size_t)po * half + h);
      } else if (!COH) {
        s_o = ld(sp_o + h);
        if (DEDUP) {
          s_n = ld(sp_n + h);
          const spn<T> sjx = ld(sp_n + nh[dx]);
#pragma unroll
          for (int d = 2; d < 6; ++d) sj[d] = ld(sp_n + nh[d]);
          sj[0] = pick(bo != 0, sjx, s_n);
          sj[1] = pick(bo != 0, s_n, sjx);
        } else {
#pragma unroll
          for (int d = 0; d < 6; ++d) sj[d] = ld(sp_n + nh[d]);
        }
      }
      if (FIRST) {
        aop.x = (h == o_half) ? (T)1 : (T)0;
        aop.y = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) { an[d].x = (nh[d] == o_half) ? (T)1 : (T)0; an[d].y = 0; }
      } else if (!DEDUP) {
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          if (COH && nb_elsewhere(nh[d])) an[d] = ld_coh(vo + (size_t)pn * half + nh[d]);
          else an[d] = ld(vo + (size_t)pn * half + nh[d]);
        }
        if (MERGE) aop = ld(vo + (size_t)pn * half + h);
      } else {
        aop = ld(vo + (size_t)pn * half + h);
        const cpx<T> anx = (COH && nb_elsewhere(nh[dx])) ? ld_coh(vo + (size_t)pn * half + nh[dx])
                                                          : ld(vo + (size_t)pn * half + nh[dx]);
#pragma unroll
        for (int d = 2; d < 6; ++d) {
          if (COH && nb_elsewhere(nh[d])) an[d] = ld_coh(vo + (size_t)pn * half + nh[d]);
          else an[d] = ld(vo + (size_t)pn * half + nh[d]);
        }
        an[0] = pick(bo != 0, anx, aop);
        an[1] = pick(bo != 0, aop, anx);
      }
      if (!FIRST) pr = NT ? ld_nt(vo + (size_t)po * half + h) : ld(vo + (size_t)po * half + h);
      if (MERGE && !FIRST) {
#pragma unroll
        for (int g = 0; g < 6; ++g) {
          if (nb_elsewhere(nhn[g])) anm[g] = vn.ld_coh((size_t)po * half + nhn[g]);
          else anm[g] = vn.ld((size_t)po * half + nhn[g]);
        }
        prevm = vn.ld((size_t)pn * half + h);
      }
      STEP_LOADS_ISSUED();
      if (COH && !FIRST) gram_rows<NW>(D, lb, s - 1, xw, gsum);   // the previous step's sums
      T ar = 0, ai = 0;
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        T hr, hi_;
        if (HOPS) {
          hr = row.v[d].x;
          hi_ = row.v[d].y;
        } else if (COH) {   // selects, not an indexed register array
          hr = po ? hp[1][d].x : hp[0][d].x;
          hi_ = po ? hp[1][d].y : hp[0][d].y;
        } else {
          hop_spinor(s_o, sj[d], hsc, hr, hi_);
        }
        cmac(hr, hi_, an[d], ar, ai);
      }
      cpx<T> ao;
      ao.x = two * ar - pr.x;
      ao.y = two * ai - pr.y;
      if (!valid) {
      } else if (NT) {
        st_nt(vo + (size_t)po * half + h, ao);
      } else {
        st(vo + (size_t)po * half + h, ao);
      }
      x[p][14] = (double)ao.x;
      x[p][15] = (double)ao.y;
    }
    // a^{n_e}_s, e = 0..5, on the n-site: the six directions in groups of
    // kGroup, each group's loads issued together (six 16-value records at
    // once are too many registers to keep the occupancy; groups of two
    // measured fastest on the HBM-resident batches).  The persistent kernel
    // runs one wave per SIMD, so registers cost it no occupancy: it takes
    // the directions in one group (FP32, loaded with the o-site's values) or
    // two (FP64).
    {
      constexpr int kGroup = COH ? (sizeof(T) == 4 ? 6 : 3) : 2;
      static_assert(kGroup >= 2, "the first group holds both x directions");
      six<T> row;
      if (HOPS) row = hrow.ld((size_t)pn * half + h);
      else if (!DEDUP && !COH) s_n = ld(sp_n + h);
      T accr[6], acci[6];
#pragma unroll
      for (int e = 0; e < 6; ++e) { accr[e] = 0; acci[e] = 0; }
      six<T> prev;
      if (!MERGE) nb6_half(h, k, bn, y, z, L, nhn);
      const int dxn = bn ? 0 : 1;   // the x direction whose neighbour is another pair
#pragma unroll
      for (int d0 = 0; d0 < 6; d0 += kGroup) {
        int nh[kGroup];
        spn<T> sj[kGroup];
        six<T> an[kGroup];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) nh[g] = nhn[d0 + g];
        if (DEDUP && !HOPS && !COH && d0 == 0) {
          const spn<T> sjx = ld(sp_o + nhn[dxn]);
          sj[0] = pick(bn != 0, sjx, s_o);
          sj[1] = pick(bn != 0, s_o, sjx);
        }
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
          if (!HOPS && !COH && (!DEDUP || d0 + g >= 2)) sj[g] = ld(sp_o + nh[g]);
          if (FIRST) {
#pragma unroll
            for (int e = 0; e < 6; ++e) {
              an[g].v[e].x = (nh[g] == sh[e]) ? (T)1 : (T)0;
              an[g].v[e].y = 0;
            }
          } else {
            if (MERGE) an[g] = anm[d0 + g];
            else if (COH && nb_elsewhere(nh[g])) an[g] = vn.ld_coh((size_t)po * half + nh[g]);
            else an[g] = vn.ld((size_t)po * half + nh[g]);
          }
        }
        if (d0 + kGroup >= 6 && !FIRST) {   // the site's own values ride with the last group
          if (MERGE) {
            prev = prevm;
          } else {
            prev = NT ? vn.ld_nt((size_t)pn * half + h) : vn.ld((size_t)pn * half + h);
            if (!DEDUP) aop = ld(vo + (size_t)pn * half + h);
          }
        }
        STEP_LOADS_ISSUED();
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
          const int d = d0 + g;
          T hr, hi_;
          if (HOPS) {
            hr = row.v[d].x;
            hi_ = row.v[d].y;
          } else if (COH) {
            hr = pn ? hp[1][d].x : hp[0][d].x;
            hi_ = pn ? hp[1][d].y : hp[0][d].y;
          } else {
            hop_spinor(s_n, sj[g], hsc, hr, hi_);
          }
#pragma unroll
          for (int e = 0; e < 6; ++e) {
            cmac(hr, hi_, an[g].v[e], accr[e], acci[e]);
          }
        }
      }
      six<T> out;
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        out.v[e].x = two * accr[e];
        out.v[e].y = two * acci[e];
        if (!FIRST) {
          out.v[e].x -= prev.v[e].x;
          out.v[e].y -= prev.v[e].y;
        }
        x[p][2 * e] = (double)out.v[e].x;
        x[p][2 * e + 1] = (double)out.v[e].y;
      }
      if (!valid) {
      } else if (NT) {
        vn.st_nt((size_t)pn * half + h, out);
      } else {
        vn.st((size_t)pn * half + h, out);
      }
      if (FIRST && valid) {   // store a_0 on the sites that hold it from now on
        st(vo + (size_t)pn * half + h, aop);
        six<T> u;
#pragma unroll
        for (int e = 0; e < 6; ++e) { u.v[e].x = (h == sh[e]) ? (T)1 : (T)0; u.v[e].y = 0; }
        vn.st((size_t)po * half + h, u);
      }
      x[p][12] = (double)aop.x;
      x[p][13] = (double)aop.y;
    }
    if (!valid)
#pragma unroll
      for (int i = 0; i < 16; ++i) x[p][i] = 0.0;
  }

  if (COH) {   // the sums of this step are formed during the next one
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 16; ++i) xw[threadIdx.x >> 6][lane][i] = x[0][i];
    arrive();
    return;
  }
  arrive();
  // Gram matrix of x over the block on the FP64 matrix core:
  // v_mfma_f64_16x16x4 with A = B = 4 columns (site pairs) of 16 components.
  // Each wave stages 16 site pairs at a time in LDS (4 rounds per PPT slice).
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      if ((lane >> 4) == rr) {
#pragma unroll
        for (int i = 0; i < 16; ++i) xs[w][lane & 15][i] = x[p][i];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double val = xs[w][4 * m + (lane >> 4)][lane & 15];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(val, val, acc, 0, 0, 0);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // result layout of v_mfma_f64_16x16x4: lane l, register r holds entry
  // (4r + l/16, l%16) of the 16x16 product
#pragma unroll
  for (int r = 0; r < 4; ++r) gsum[w][(4 * r + (lane >> 4)) * 16 + (lane & 15)] = acc[r];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kNP)
    D.part[((size_t)(s - 1) * kNP + t) * D.nblk + lb] = gram_combo<NW>(gsum, gram_combo_index(t));
}

// Step s with two site pairs of one y column per thread (7-vector form, FP32,
// hoppings recomputed, launched kernels with two pairs per thread): thread j
// of a chain takes half-row index k in rows 2 (j / (L/2)) and the next one of
// one z-plane.  As in the pair kernel's column form, the y + 1 neighbour of
// the first pair's o-site is the second pair's n-site and the y + 1
// neighbour of its n-site is the second pair's o-site (and the same for
// y - 1 from the second pair): those spinors, the n-site's a^o_{s-1} and the
// o-site's six a^n_{s-1} come from the thread's own loads, so two pairs load
// 68 values instead of 78.  Every site's sums run over the six directions in
// the same order as in step_block, so the vector values agree with it bit
// for bit; the n-site's loads are issued by direction group (x, y, z) for
// both pairs together.
template <typename T>
__device__ inline six<T> pick6(bool c, const six<T>& a, const six<T>& b) {
  six<T> r;
#pragma unroll
  for (int e = 0; e < 6; ++e) r.v[e] = pick(c, a.v[e], b.v[e]);
  return r;
}

template <typename T, bool FIRST, bool NT, int BT>
__device__ __forceinline__ void step_block_col2(const Desc& D, const int lb, const int s,
                                                double (*xs)[16][17], double (*gsum)[256]) {
  constexpr int NW = BT / 64;
  const int L = D.L, half = D.half, hx = L >> 1;
  const Ctl* ctl = D.ctl;
  const int pO = ctl->parity_o;
  const int po = pO ^ (s & 1);          // parity of the sites that carry a^o_s
  const int pn = po ^ 1;                // parity of the sites that carry a^n_s
  const int o_half = ctl->o_half;
  int sh[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) sh[e] = FIRST ? ctl->start_half[1 + e] : 0;
  const double hsc = -D.t / D.a;        // Ht = -(t/a) t_ij
  const T two = FIRST ? (T)1 : (T)2;     // |a_1> = Ht|a_0>, then 2 Ht|a_{s-1}> - |a_{s-2}>
  const GLOBAL spn<T>* sp = (const GLOBAL spn<T>*)D.spin;            // [2][half]
  GLOBAL cpx<T>* vo = (GLOBAL cpx<T>*)D.vec;                         // o-slots [2][half]
  const Planes<T> vn = planes<T>((cpx<T>*)D.vec + D.N, D.N);        // n-slots [2][half]
  const GLOBAL spn<T>* sp_o = sp + (size_t)po * half;
  const GLOBAL spn<T>* sp_n = sp + (size_t)pn * half;
  auto ind = [&](int hh) {   // a^o_0 = |o> at half-row index hh (o's parity)
    cpx<T> r;
    r.x = (hh == o_half) ? (T)1 : (T)0;
    r.y = 0;
    return r;
  };
  auto ind6 = [&](int hh) {   // a^{n_e}_0 = |n_e> at half-row index hh
    six<T> r;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      r.v[e].x = (hh == sh[e]) ? (T)1 : (T)0;
      r.v[e].y = 0;
    }
    return r;
  };
  double x[2][16];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int i = 0; i < 16; ++i) x[q][i] = 0.0;
  const int j = lb * BT + (int)threadIdx.x;
  if (j < half / 2) {
    const int r = (int)fdiv((uint32_t)j, D.div_hx);
    const int k = j - r * hx;
    const int R = 2 * r;   // row index y + L z of the first pair
    const int z = (int)fdiv((uint32_t)R, D.div_L);
    const int y0 = R - z * L;
    const int h0 = R * hx + k;
    const int b0 = (y0 + z + po) & 1;   // x = 2k + b of the first pair's o-site
    spn<T> so[2], sn[2];   // the pairs' own spinors
    cpx<T> aop[2];         // a^o_{s-1} at the n-sites
    {   // a^o_s on the o-sites
      int nh[2][6];
      spn<T> sjx[2], sj[2][6];
      cpx<T> anx[2], an[2][6], pr[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int h = h0 + q * hx, bo = b0 ^ q;
        nb6_half(h, k, bo, y0 + q, z, L, nh[q]);
        const int nx = bo ? nh[q][0] : nh[q][1];   // the x neighbour that is another pair
        so[q] = ld(sp_o + h);
        sn[q] = ld(sp_n + h);
        sjx[q] = ld(sp_n + nx);
        if (FIRST) {
          aop[q] = ind(h);
          anx[q] = ind(nx);
        } else {
          aop[q] = ld(vo + (size_t)pn * half + h);
          anx[q] = ld(vo + (size_t)pn * half + nx);
        }
#pragma unroll
        for (int d = 2; d < 6; ++d) {
          if ((d == 2 && q == 0) || (d == 3 && q == 1)) continue;   // inside the column
          sj[q][d] = ld(sp_n + nh[q][d]);
          an[q][d] = FIRST ? ind(nh[q][d]) : ld(vo + (size_t)pn * half + nh[q][d]);
        }
        pr[q].x = 0;
        pr[q].y = 0;
        if (!FIRST) pr[q] = NT ? ld_nt(vo + (size_t)po * half + h) : ld(vo + (size_t)po * half + h);
      }
      STEP_LOADS_ISSUED();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int h = h0 + q * hx, bo = b0 ^ q;
        sj[q][0] = pick(bo != 0, sjx[q], sn[q]);
        sj[q][1] = pick(bo != 0, sn[q], sjx[q]);
        an[q][0] = pick(bo != 0, anx[q], aop[q]);
        an[q][1] = pick(bo != 0, aop[q], anx[q]);
        if (q == 0) {
          sj[0][2] = sn[1];
          an[0][2] = aop[1];
        } else {
          sj[1][3] = sn[0];
          an[1][3] = aop[0];
        }
        T ar = 0, ai = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          T hr, hi_;
          hop_spinor(so[q], sj[q][d], hsc, hr, hi_);
          cmac(hr, hi_, an[q][d], ar, ai);
        }
        cpx<T> ao;
        ao.x = two * ar - pr[q].x;
        ao.y = two * ai - pr[q].y;
        if (NT) st_nt(vo + (size_t)po * half + h, ao);
        else st(vo + (size_t)po * half + h, ao);
        x[q][14] = (double)ao.x;
        x[q][15] = (double)ao.y;
      }
    }
    {   // a^{n_e}_s, e = 0..5, on the n-sites: x, y and z directions in turn
      int nhn[2][6];
#pragma unroll
      for (int q = 0; q < 2; ++q) nb6_half(h0 + q * hx, k, b0 ^ q ^ 1, y0 + q, z, L, nhn[q]);
      T accr[2][6], acci[2][6];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 6; ++e) {
          accr[q][e] = 0;
          acci[q][e] = 0;
        }
      auto acc6 = [&](int q, const spn<T>& sj, const six<T>& a6) {
        T hr, hi_;
        hop_spinor(sn[q], sj, hsc, hr, hi_);
#pragma unroll
        for (int e = 0; e < 6; ++e) cmac(hr, hi_, a6.v[e], accr[q][e], acci[q][e]);
      };
      six<T> own6[2];   // a^n_{s-1} at the pairs' own o-sites
      {   // x: the pair's own o-site and the neighbour in the next or previous pair
        spn<T> sjx[2];
        six<T> anx6[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int h = h0 + q * hx, bn = b0 ^ q ^ 1;
          const int nx = bn ? nhn[q][0] : nhn[q][1];
          sjx[q] = ld(sp_o + nx);
          own6[q] = FIRST ? ind6(h) : vn.ld((size_t)po * half + h);
          anx6[q] = FIRST ? ind6(nx) : vn.ld((size_t)po * half + nx);
        }
        STEP_LOADS_ISSUED();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const bool bn = (b0 ^ q ^ 1) != 0;
          acc6(q, pick(bn, sjx[q], so[q]), pick6(bn, anx6[q], own6[q]));   // x + 1
          acc6(q, pick(bn, so[q], sjx[q]), pick6(bn, own6[q], anx6[q]));   // x - 1
        }
      }
      {   // y: one neighbour is the other pair's o-site
        spn<T> sjy[2];
        six<T> any6[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int ny = nhn[q][q == 0 ? 3 : 2];   // the y neighbour outside the column
          sjy[q] = ld(sp_o + ny);
          any6[q] = FIRST ? ind6(ny) : vn.ld((size_t)po * half + ny);
        }
        STEP_LOADS_ISSUED();
        acc6(0, so[1], own6[1]);     // y + 1
        acc6(0, sjy[0], any6[0]);    // y - 1
        acc6(1, sjy[1], any6[1]);    // y + 1
        acc6(1, so[0], own6[0]);     // y - 1
      }
      six<T> prev[2];
      {   // z, and the sites' own a^n_{s-2}
        spn<T> sjz[2][2];
        six<T> anz6[2][2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int h = h0 + q * hx;
#pragma unroll
          for (int g = 0; g < 2; ++g) {
            sjz[q][g] = ld(sp_o + nhn[q][4 + g]);
            anz6[q][g] = FIRST ? ind6(nhn[q][4 + g]) : vn.ld((size_t)po * half + nhn[q][4 + g]);
          }
          if (!FIRST)
            prev[q] = NT ? vn.ld_nt((size_t)pn * half + h) : vn.ld((size_t)pn * half + h);
        }
        STEP_LOADS_ISSUED();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          acc6(q, sjz[q][0], anz6[q][0]);
          acc6(q, sjz[q][1], anz6[q][1]);
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int h = h0 + q * hx;
        six<T> out;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
          out.v[e].x = two * accr[q][e];
          out.v[e].y = two * acci[q][e];
          if (!FIRST) {
            out.v[e].x -= prev[q].v[e].x;
            out.v[e].y -= prev[q].v[e].y;
          }
          x[q][2 * e] = (double)out.v[e].x;
          x[q][2 * e + 1] = (double)out.v[e].y;
        }
        if (NT) vn.st_nt((size_t)pn * half + h, out);
        else vn.st((size_t)pn * half + h, out);
        if (FIRST) {   // store a_0 on the sites that hold it from now on
          st(vo + (size_t)pn * half + h, aop[q]);
          vn.st((size_t)po * half + h, ind6(h));
        }
        x[q][12] = (double)aop[q].x;
        x[q][13] = (double)aop[q].y;
      }
    }
  }
  gram_staged<2, NW>(D, lb, s, x, xs, gsum);
}

// The column form (two site pairs per thread, FP32) is held to three waves per
// SIMD (159 VGPRs; left to itself the compiler takes 172 and two waves, and
// the 64 x 32^3 round takes 35.4 us instead of 32.1).
template <typename T, bool FIRST, int PPT, bool HOPS, bool NT, int BT = kStepThreads>
__global__ __launch_bounds__(BT)
__attribute__((amdgpu_waves_per_eu(PPT == 2 && !HOPS && sizeof(T) == 4 ? 3 : 1))) void k_step(
    const Desc* __restrict__ descs, const int* __restrict__ blkoff, int nact, int s_arg,
    const int* __restrict__ act_end) {
  __shared__ double xs[BT / 64][16][17];
  __shared__ double gsum[BT / 64][256];
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  int c = 0;
  {
    int lo = 0, hi = nact - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (blkoff[mid] <= gb) lo = mid; else hi = mid - 1;
    }
    c = lo;
  }
  const Desc& D = descs[c];
  const int s = chain_step(s_arg, act_end, c, D.S);
  if (s == 0) return;   // uniform over the block: the chain does not step now
  if constexpr (PPT == 2 && !HOPS && sizeof(T) == 4)
    step_block_col2<T, FIRST, NT, BT>(D, gb - blkoff[c], s, xs, gsum);
  else
    step_block<T, FIRST, PPT, HOPS, NT, false, NoArrive, BT>(D, gb - blkoff[c], s, xs, gsum);
}

// ------------------------------------------- persistent single chain ---
// A lone mid-size chain (its vectors fit one compute die's L2) takes all M/2
// steps of a proposal in one launch instead of M/2 launches of a few
// microseconds each.  Blocks are dealt to the eight compute dies (XCDs) in
// turn; the first block to start claims its die, and the first nb blocks on
// that die take the work (the others return), so every block of the run
// shares one L2 and the step barrier's counter lives there.  That L2 is the
// point of coherence for all of them, so a step's stores are visible to the
// other blocks once they have completed (the vector L1 writes through): each
// wave waits for its stores, one thread per block counts in at the L2 and
// polls it, and the next step reads the neighbour values that other blocks
// stored with device-scope loads, which skip the compute unit's L1 and are
// served by the L2; values this block stored (through the same L1) and the
// spinors, fixed during a proposal, load as usual.  (Reading every
// neighbour past the L1 sent the stencil's reuse, six loads per value, to
// the L2 through the links of the few compute units a lone chain uses.)  No cache is written
// back or invalidated: the device-scope fences that would (the L2 write-back
// for other dies, the L1 and L2 invalidation) cost more per step than a
// kernel launch, for visibility this run never needs.  Waits are
// bounded: on a
// timeout the run sets an error flag, every block returns, and the
// reconstruction leaves the chain unchanged.
constexpr int kBarrierSpins = 1 << 21;

__device__ inline unsigned xcd_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 0xfu;   // HW_REG_XCC_ID, bits 3:0
}

// The step barrier in two phases.  Arrive: every wave waits for its stores
// of the step (they are then in the L2), and one thread counts the block in.
// Wait: that thread polls the count, and the block proceeds once every block
// of the run has arrived.  Between the two the block forms its Gram sums,
// which no other block reads.
struct DieArrive {
  unsigned* count;
  __device__ void operator()() const {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached the L2
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

__device__ inline bool die_wait(unsigned* count, unsigned target, unsigned* err, int* ok_sh) {
  if (threadIdx.x == 0) {
    int ok = 1;
    for (int i = 0;
         __hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++i) {
      // another block's time-out is checked every 64th poll (one load per poll)
      if (i >= kBarrierSpins ||
          ((i & 63) == 63 &&
           __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u)) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    *ok_sh = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return *ok_sh != 0;
}

template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_persist(const Desc* __restrict__ descs, int nb) {
  constexpr int NW = BT / 64;
  __shared__ double xw[NW][64][17];   // each thread's 16 values of the last step
  __shared__ double gsum[NW][256];
  __shared__ int tk, ok_sh;
  const Desc& D = descs[0];
  unsigned* bar = D.ctl->bar;
  if (threadIdx.x == 0) {
    const unsigned x = xcd_id() + 1u;
    unsigned old = 0u;
    __hip_atomic_compare_exchange_strong(&bar[1], &old, x, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_SYSTEM);
    const unsigned die = old ? old : x;   // old == 0: this block claimed its die
    tk = (x == die) ? (int)__hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM)
                    : nb;
  }
  __syncthreads();
  const int lb = tk;
  if (lb >= nb) return;
  // the twelve hopping amplitudes of this thread's site pair, fixed for the
  // proposal: hp[q][d] from the site of parity q to its neighbour d
  cpx<T> hp[2][6];
  {
    const int h = lb * BT + (int)threadIdx.x;
    const int hh = h < D.half ? h : 0;   // threads past the lattice take none
    int k, y, z;
    split_half(hh, D, k, y, z);
    const GLOBAL spn<T>* sp = (const GLOBAL spn<T>*)D.spin;
    const double hsc = -D.t / D.a;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int nh[6];
      nb6_half(hh, k, (y + z + q) & 1, y, z, D.L, nh);
      const spn<T> si = ld(sp + (size_t)q * D.half + hh);
#pragma unroll
      for (int d = 0; d < 6; ++d)
        hop_spinor(si, ld(sp + (size_t)(q ^ 1) * D.half + nh[d]), hsc, hp[q][d].x, hp[q][d].y);
    }
  }
  const DieArrive arrive{&bar[2]};
  for (int s = 1; s <= D.S; ++s) {
    if (s == 1)
      step_block<T, true, 1, false, false, true, DieArrive, BT>(D, lb, 1, nullptr, gsum, arrive, hp,
                                                                xw);
    else
      step_block<T, false, 1, false, false, true, DieArrive, BT>(D, lb, s, nullptr, gsum, arrive,
                                                                 hp, xw);
    if (s == D.S) break;
    if (!die_wait(&bar[2], (unsigned)nb * (unsigned)s, &bar[3], &ok_sh)) return;
  }
  gram_rows<NW>(D, lb, D.S, xw, gsum);   // the last step's sums
}

// Census of the dies a grid of `blocks` lands on: counts[die] += 1 per block.
__global__ void k_die_census(unsigned* counts) {
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(&counts[xcd_id()], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Small lattices: one workgroup runs all M/2 steps of one chain out of LDS,
// so a proposal costs one launch instead of M/2.  Same arithmetic as k_step
// (sum over the six directions in order, a_{s+1} over a_{s-1} in place, the
// same 49 Gram sums per step on the FP64 matrix core), organised for latency
// rather than bandwidth, since a small lattice gives a step only a few
// hundred site pairs:
//  * the hopping amplitudes t_{i, n_d(i)} and the neighbours' half-row
//    indices are tabulated once per proposal (the spins do not change within
//    one), so a step reads them instead of recomputing them;
//  * a step is 7 x half independent items (vector j, site pair h) spread over
//    all threads, each a six-term sum, instead of one thread forming all
//    seven vectors of a site pair in sequence;
//  * the Gram operands are read straight from the LDS planes.
// LDS planes (index par * half + h for parity par, half-row index h):
//   hp[d]  t_{i, n_d(i)} of site i = (par, h), d = 0..5
//   vo     the o-vector slot,  vn[e] the slot of neighbour vector e = 0..5
//   nb[d]  half-row index of n_d(i) (parity par ^ 1)
// 13 complex values and 6 indices per site: 128 B (FP32), 232 B (FP64).
template <typename T>
__global__ __launch_bounds__(kResThreads) void k_resident(const Desc* __restrict__ descs) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ double gsum[2][4][256];   // double-buffered by step parity
  const Desc& D = descs[blockIdx.x];
  const int L = D.L, hx = L >> 1, half = D.half, N = D.N;
  cpx<T>* hp = (cpx<T>*)smem;                 // [6][2][half]
  cpx<T>* vo = hp + 6 * N;                    // [2][half]
  cpx<T>* vn = vo + N;                        // [6][2][half]
  int* nb = (int*)(vn + 6 * N);               // [6][2][half]
  const Ctl* ctl = D.ctl;
  const int pO = ctl->parity_o, o_half = ctl->o_half;
  int sh[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) sh[e] = ctl->start_half[1 + e];
  const GLOBAL spn<T>* gsp = (const GLOBAL spn<T>*)D.spin;
  const double hsc = -D.t / D.a;   // Ht = -(t/a) t_ij
  // global (not flat) stores of the step partials: a flat store counts against
  // the LDS wait counter, so every barrier would wait for its write to memory
  GLOBAL double* part = (GLOBAL double*)D.part;

  // tables, and the start vectors a_0 = e_o (o-slots, parity of o) and
  // e_{n_e} (n-slots, the other parity); every other slot starts at zero
  for (int q = threadIdx.x; q < N; q += kResThreads) {
    const int par = (q >= half) ? 1 : 0, h = q - par * half;
    const int k = h % hx, r = h / hx, y = r % L, z = r / L;
    const int x = 2 * k + ((y + z + par) & 1);
    const spn<T> si = ld(gsp + q);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int nh = nb_half(x, y, z, d, L);
      T hr, hi_;
      hop_spinor(si, ld(gsp + (size_t)(par ^ 1) * half + nh), hsc, hr, hi_);
      hp[d * N + q] = cpx<T>{hr, hi_};
      nb[d * N + q] = nh;
      vn[d * N + q] = cpx<T>{(par != pO && h == sh[d]) ? (T)1 : (T)0, (T)0};
    }
    vo[q] = cpx<T>{(par == pO && h == o_half) ? (T)1 : (T)0, (T)0};
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int items = 7 * half, chunks = (half + 3) >> 2;
  const float inv_half = 1.0f / (float)half;
  // two barriers per step: after the items (the Gram reads see them) and after
  // the Gram sums (the next step may overwrite what they read, and its
  // combination of the sums reads them)
  __syncthreads();
  // On the smallest lattices (at most half the threads have an item) the 49
  // block sums of step s are formed by the last wave, which has no item,
  // during the items of step s + 1, from the other gsum buffer: off the
  // critical path of a step that is mostly latency.  Otherwise the first 49
  // threads form them right after the Gram sums.
  const bool defer = items <= kResThreads / 2;
  const int t49 = defer ? (int)threadIdx.x - (kResThreads - 64) : (int)threadIdx.x;
  const bool combiner = t49 >= 0 && t49 < kNP;
  const Combo cmb = gram_combo_index(combiner ? t49 : 0);
  for (int s = 1; s <= D.S; ++s) {
    if (defer && s > 1 && combiner)
      part[(size_t)(s - 2) * kNP + t49] = gram_combo(gsum[(s - 1) & 1], cmb);
    const int po = pO ^ (s & 1), pn = po ^ 1;   // parities that carry a^o_s, a^n_s
    const T two = (s == 1) ? (T)1 : (T)2;   // |a_1> = Ht|a_0>, then 2 Ht|a_{s-1}> - |a_{s-2}>
    // item (j, h): j = 0 forms a^o_s at the o-site (po, h), j >= 1 forms
    // a^{n_{j-1}}_s at the n-site (pn, h); at s = 1 the slot being
    // overwritten holds zero, so subtracting it is exact
    for (int q = threadIdx.x; q < items; q += kResThreads) {
      const int j = (int)(((float)q + 0.5f) * inv_half), h = q - j * half;
      const int par = j ? pn : po;
      const int row = par * half + h;
      const cpx<T>* src = j ? vn + (size_t)(j - 1) * N + (par ^ 1) * half : vo + (par ^ 1) * half;
      cpx<T>* dst = (j ? vn + (size_t)(j - 1) * N : vo) + row;
      int nh[6];
      cpx<T> hv[6], an[6];
#pragma unroll
      for (int d = 0; d < 6; ++d) nh[d] = nb[d * N + row];
#pragma unroll
      for (int d = 0; d < 6; ++d) hv[d] = hp[d * N + row];
      const cpx<T> pr = *dst;
#pragma unroll
      for (int d = 0; d < 6; ++d) an[d] = src[nh[d]];
      // every load of the item is issued before the arithmetic: two LDS round
      // trips (indices, then values) instead of one per direction
      __builtin_amdgcn_sched_barrier(0);
      T ar = 0, ai = 0;
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        cmac(hv[d].x, hv[d].y, an[d], ar, ai);
      }
      *dst = cpx<T>{two * ar - pr.x, two * ai - pr.y};
    }
    __syncthreads();
    // Gram matrix of the 16-vector of every site pair h,
    //   (Re/Im a^{n_0..5}_s at (pn, h), Re/Im a^o_{s-1} at (pn, h), Re/Im a^o_s at (po, h)),
    // on the FP64 matrix core: v_mfma_f64_16x16x4 with A = B, four site pairs
    // per instruction (lane: component lane % 16 of pair lane / 16)
    d4v acc = {0.0, 0.0, 0.0, 0.0};
    if (w < 4) {   // the first four waves
      const int comp = lane & 15;
      const T* base = (const T*)((comp < 12) ? vn + (size_t)(comp >> 1) * N + pn * half
                                              : vo + ((comp < 14) ? pn : po) * half) + (comp & 1);
      // four chunks of four site pairs per round, loads ahead of the products
      for (int c0 = w; c0 < chunks; c0 += 16) {
        double val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int h = 4 * (c0 + 4 * u) + (lane >> 4);
          const double v = (double)base[2 * min(h, half - 1)];   // unconditional load
          val[u] = (h < half) ? v : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(val[u], val[u], acc, 0, 0, 0);
      }
    }
    // result layout of v_mfma_f64_16x16x4: lane l, register r holds entry
    // (4r + l/16, l%16) of the 16x16 product
    if (w < 4) {
#pragma unroll
      for (int r = 0; r < 4; ++r) gsum[s & 1][w][(4 * r + (lane >> 4)) * 16 + (lane & 15)] = acc[r];
    }
    __syncthreads();
    if (!defer && combiner) part[(size_t)(s - 1) * kNP + t49] = gram_combo(gsum[s & 1], cmb);
  }
  if (defer && combiner) part[(size_t)(D.S - 1) * kNP + t49] = gram_combo(gsum[D.S & 1], cmb);
}

// Neumaier-compensated sum helper: (sum, comp) += v.
__device__ inline void nsum(double& sum, double& comp, double v) {
  const double tt = sum + v;
  comp += (fabs(sum) >= fabs(v)) ? (sum - tt) + v : (v - tt) + sum;
  sum = tt;
}

// Sum of one contiguous run of block partials, in block order, with
// Neumaier compensation (two-double loads, eight in flight).
__device__ inline double sum_run(const double* __restrict__ src, int n) {
  double sum = 0.0, comp = 0.0;
  int b = 0;
  if ((((uintptr_t)src) & 15) == 0) {
    const double2* s2 = (const double2*)src;
    for (; b + 16 <= n; b += 16) {
      double2 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = s2[(b >> 1) + i];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        nsum(sum, comp, v[i].x);
        nsum(sum, comp, v[i].y);
      }
    }
  }
  for (; b < n; ++b) nsum(sum, comp, src[b]);
  return sum + comp;
}

// The pair form {|o>, |v>}: |a^o_0> = |o>, |a^v_0> = |v> = sum_d delta_d |n_d>
// (|v> = Delta|o>, Section 2.2).  Same bipartite storage as above with one
// v-slot in place of the six n-slots: a^o_s lives on parity p(o)^(s&1), a^v_s
// on the other.  Per step the block sums P^{oo}_s = <a^o_s|a^o_s>,
// P^{vv}_s = <a^v_s|a^v_s> and Q^{ov}_s = <a^o_{s-1}|a^v_s> (4 real numbers;
// the pairs that vanish on a bipartite lattice are not formed) with wavefront
// shuffles and one LDS step.
//   A thread takes YP site pairs of one column: the same half-row index k in
// rows y0 .. y0 + YP - 1 of one z-plane (y0 a multiple of YP; thread j of a
// chain takes rows YP (j / (L/2)) onward, so the threads of a wave cover whole
// row segments).  The pair's two sites alternate between the x offsets of a
// row, so the y+1 neighbour of a pair's o-site is the next pair's v-site and
// the y+1 neighbour of its v-site is the next pair's o-site (and the same for
// y-1): inside a column those spinors and values come from the thread's own
// loads.  A pair alone loads 26 values (own spinors, values and the x
// neighbour that is the pair's other site shared as well); two pairs of a
// column load 44.  Every site's sum runs over the six directions in the same
// order as the other kernels, so the vector values do not depend on YP.
template <typename T, bool FIRST, int YP>
__global__ __launch_bounds__(kStepThreads) void k_step_ov(const Desc* __restrict__ descs,
                                                          const int* __restrict__ blkoff,
                                                          int nact, int s_arg,
                                                          const int* __restrict__ act_end) {
  __shared__ double red[kStepWaves][kNP2];
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  int c = 0;
  {
    int lo = 0, hi = nact - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (blkoff[mid] <= gb) lo = mid; else hi = mid - 1;
    }
    c = lo;
  }
  const Desc& D = descs[c];
  const int s = chain_step(s_arg, act_end, c, D.S);
  if (s == 0) return;   // uniform over the block: the chain does not step now
  const int lb = gb - blkoff[c];
  const int L = D.L, half = D.half, hx = L >> 1;
  const Ctl* ctl = D.ctl;
  const int pO = ctl->parity_o;
  const int po = pO ^ (s & 1);          // parity of the sites that carry a^o_s
  const int pn = po ^ 1;                // parity of the sites that carry a^v_s
  const int o_half = ctl->o_half;
  int sh[6];
  T dr[6], di[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    sh[e] = FIRST ? ctl->start_half[1 + e] : 0;
    dr[e] = FIRST ? (T)ctl->delta[2 * e] : (T)0;
    di[e] = FIRST ? (T)ctl->delta[2 * e + 1] : (T)0;
  }
  const double hsc = -D.t / D.a;        // Ht = -(t/a) t_ij
  const T two = FIRST ? (T)1 : (T)2;     // |a_1> = Ht|a_0>, then 2 Ht|a_{s-1}> - |a_{s-2}>
  const GLOBAL spn<T>* sp = (const GLOBAL spn<T>*)D.spin;
  GLOBAL cpx<T>* vo = (GLOBAL cpx<T>*)D.vec;               // o-slots [2][half]
  GLOBAL cpx<T>* vv = (GLOBAL cpx<T>*)D.vec + D.N;         // v-slots [2][half]
  const GLOBAL spn<T>* sp_o = sp + (size_t)po * half;
  const GLOBAL spn<T>* sp_n = sp + (size_t)pn * half;
  // a^v_0 at a site with half-row index hh on the parity of o's neighbours
  auto v0 = [&](int hh) {
    cpx<T> r = {(T)0, (T)0};
#pragma unroll
    for (int e = 0; e < 6; ++e)
      if (hh == sh[e]) { r.x += dr[e]; r.y += di[e]; }
    return r;
  };
  auto ind = [&](int hh) {   // a^o_0 = |o> at half-row index hh (o's parity)
    cpx<T> r;
    r.x = (hh == o_half) ? (T)1 : (T)0;
    r.y = 0;
    return r;
  };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int j = lb * kStepThreads + (int)threadIdx.x;
  if (j < half / YP) {
    int k, y0, z, h0;
    if (YP == 1) {
      split_half(j, D, k, y0, z);
      h0 = j;
    } else {
      const int r = (int)fdiv((uint32_t)j, D.div_hx);
      k = j - r * hx;
      const int R = r * YP;   // row index y + L z of the column's first pair
      z = (int)fdiv((uint32_t)R, D.div_L);
      y0 = R - z * L;
      h0 = R * hx + k;
    }
    const int b0 = (y0 + z + po) & 1;   // x = 2k + b of the first pair's o-site
    // Each phase's loads are issued together, before its arithmetic (one
    // memory round trip per phase; issuing both phases' loads at once
    // measured no faster in FP32 and slower in FP64, whose registers then
    // halve the occupancy).
    spn<T> sio[YP], siv[YP];
    cpx<T> aop[YP], anh[YP], ao[YP], av[YP];
    {   // a^o_s on the o-sites
      int nh[YP][6];
      spn<T> sj[YP][6], sjx[YP];
      cpx<T> an[YP][6], anx[YP], pr[YP];
#pragma unroll
      for (int q = 0; q < YP; ++q) {
        const int h = h0 + q * hx, bo = b0 ^ (q & 1);
        nb6_half(h, k, bo, y0 + q, z, L, nh[q]);
        const int nx = bo ? nh[q][0] : nh[q][1];   // the x neighbour that is another pair
        sio[q] = ld(sp_o + h);
        siv[q] = ld(sp_n + h);
        sjx[q] = ld(sp_n + nx);
        if (FIRST) {
          aop[q] = ind(h);
          anx[q] = ind(nx);
        } else {
          aop[q] = ld(vo + (size_t)pn * half + h);
          anx[q] = ld(vo + (size_t)pn * half + nx);
        }
#pragma unroll
        for (int d = 2; d < 6; ++d) {
          if ((d == 2 && q + 1 < YP) || (d == 3 && q > 0)) continue;   // inside the column
          sj[q][d] = ld(sp_n + nh[q][d]);
          an[q][d] = FIRST ? ind(nh[q][d]) : ld(vo + (size_t)pn * half + nh[q][d]);
        }
        pr[q].x = 0;
        pr[q].y = 0;
        if (!FIRST) pr[q] = ld(vo + (size_t)po * half + h);
      }
      STEP_LOADS_ISSUED();
#pragma unroll
      for (int q = 0; q < YP; ++q) {
        const int h = h0 + q * hx, bo = b0 ^ (q & 1);
        // the other x direction's neighbour is the pair's own v-site
        sj[q][0] = pick(bo, sjx[q], siv[q]);
        sj[q][1] = pick(bo, siv[q], sjx[q]);
        an[q][0] = pick(bo, anx[q], aop[q]);
        an[q][1] = pick(bo, aop[q], anx[q]);
        if (q + 1 < YP) { sj[q][2] = siv[q + 1]; an[q][2] = aop[q + 1]; }
        if (q > 0) { sj[q][3] = siv[q - 1]; an[q][3] = aop[q - 1]; }
        T ar = 0, ai = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          T hr, hi_;
          hop_spinor(sio[q], sj[q][d], hsc, hr, hi_);
          cmac(hr, hi_, an[q][d], ar, ai);
        }
        ao[q].x = two * ar - pr[q].x;
        ao[q].y = two * ai - pr[q].y;
        st(vo + (size_t)po * half + h, ao[q]);
      }
    }
    {   // a^v_s on the v-sites
      int nh[YP][6];
      spn<T> sj[YP][6], sjx[YP];
      cpx<T> an[YP][6], anx[YP], pr[YP];
#pragma unroll
      for (int q = 0; q < YP; ++q) {
        const int h = h0 + q * hx, bn = b0 ^ (q & 1) ^ 1;
        nb6_half(h, k, bn, y0 + q, z, L, nh[q]);
        const int nx = bn ? nh[q][0] : nh[q][1];
        sjx[q] = ld(sp_o + nx);
        if (FIRST) {
          anh[q] = v0(h);
          anx[q] = v0(nx);
        } else {
          anh[q] = ld(vv + (size_t)po * half + h);
          anx[q] = ld(vv + (size_t)po * half + nx);
        }
#pragma unroll
        for (int d = 2; d < 6; ++d) {
          if ((d == 2 && q + 1 < YP) || (d == 3 && q > 0)) continue;
          sj[q][d] = ld(sp_o + nh[q][d]);
          an[q][d] = FIRST ? v0(nh[q][d]) : ld(vv + (size_t)po * half + nh[q][d]);
        }
        pr[q].x = 0;
        pr[q].y = 0;
        if (!FIRST) pr[q] = ld(vv + (size_t)pn * half + h);
      }
      STEP_LOADS_ISSUED();
#pragma unroll
      for (int q = 0; q < YP; ++q) {
        const int h = h0 + q * hx, bn = b0 ^ (q & 1) ^ 1;
        sj[q][0] = pick(bn, sjx[q], sio[q]);
        sj[q][1] = pick(bn, sio[q], sjx[q]);
        an[q][0] = pick(bn, anx[q], anh[q]);
        an[q][1] = pick(bn, anh[q], anx[q]);
        if (q + 1 < YP) { sj[q][2] = sio[q + 1]; an[q][2] = anh[q + 1]; }
        if (q > 0) { sj[q][3] = sio[q - 1]; an[q][3] = anh[q - 1]; }
        T ar = 0, ai = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          T hr, hi_;
          hop_spinor(siv[q], sj[q][d], hsc, hr, hi_);
          cmac(hr, hi_, an[q][d], ar, ai);
        }
        av[q].x = two * ar - pr[q].x;
        av[q].y = two * ai - pr[q].y;
        st(vv + (size_t)pn * half + h, av[q]);
        if (FIRST) {
          st(vo + (size_t)pn * half + h, aop[q]);
          st(vv + (size_t)po * half + h, anh[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < YP; ++q) {
      const double aor = ao[q].x, aoi = ao[q].y, avr = av[q].x, avi = av[q].y;
      const double apr = aop[q].x, api = aop[q].y;
      acc[0] += aor * aor + aoi * aoi;
      acc[1] += avr * avr + avi * avi;
      acc[2] += apr * avr + api * avi;
      acc[3] += apr * avi - api * avr;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_xor(acc[v], off);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[w][v] = acc[v];
  __syncthreads();
  if (threadIdx.x < kNP2) {
    const int t = threadIdx.x;
    double r = red[0][t];
#pragma unroll
    for (int w = 1; w < kStepWaves; ++w) r += red[w][t];
    D.part[((size_t)(s - 1) * kNP2 + t) * D.nblk + lb] = r;
  }
}

// ------------------------------------------------ pair form, two steps ---
// Steps s and s + 1 (s >= 2) of the pair form in one launch.  A block takes
// a tile of ty x tz full x-rows of one chain.  Step s + 1 on the tile needs
// step s on the tile and on one row around it, which needs the stored values
// two rows out, so the block stages the tile with two halo rows on each side
// in y and z (o-slot, v-slot and spinor of every site) in LDS, advances the
// inner region by step s and the tile by step s + 1 there, and writes the
// tile's slots back.  Per site and two steps that is 16 B of slots and 16 B
// of spinor read and 16 B written (FP32), against 2 x 40 B for two one-step
// launches; the halo rows are read again by the neighbouring tiles, mostly
// from the L2 and the last-level cache.  The advance is k_step_ov's, term for
// term (same neighbour order, hopping and fused products), so every vector
// value agrees bit for bit with the one-step kernel; the block sums of a step
// run over the tile's own sites, and the partial-sum slots of a chain beyond
// its tile count are written as zeros.
//
// Tile-local site index: i = (lz * (ty + 4) + ly) * L + x, ly and lz the
// staged row (halo included), so y neighbours are i +- L and z neighbours
// i +- (ty + 4) L; x wraps within the row.  The tile origin (y0, z0) is a
// multiple of the (even) tile size, so a staged site's parity is
// (x + ly + lz) & 1, its global one.
template <typename T>
__device__ inline cpx<T> tile_advance(const cpx<T>* X, const spn<T>* S, int i, int x, int L,
                                      int zs, double hsc) {
  const int nb[6] = {(x + 1 == L) ? i + 1 - L : i + 1, (x == 0) ? i + L - 1 : i - 1,
                     i + L, i - L, i + zs, i - zs};
  const spn<T> si = S[i];
  T ar = 0, ai = 0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    T hr, hi_;
    hop_spinor(si, S[nb[d]], hsc, hr, hi_);
    cmac(hr, hi_, X[nb[d]], ar, ai);
  }
  const cpx<T> pr = X[i];
  return cpx<T>{(T)2 * ar - pr.x, (T)2 * ai - pr.y};
}

// One step over staged rows ly in [r0, ty + 4 - r0), lz in [r0, tz + 4 - r0)
// (r0 = 1: the tile and one row around it; r0 = 2: the tile), in place: a
// site of the parity that carries a^o_s advances its o-slot, a site of the
// other parity its v-slot, and neither slot is read at that parity during the
// step.  Sums over the tile's own sites: g[0] = |a^o_s|^2, g[1] = |a^v_s|^2,
// g[2] + i g[3] = conj(a^o_{s-1}) a^v_s (a^o_{s-1} is the o-slot of the
// v-site, not advanced in this step).
template <typename T>
__device__ inline void tile_step(cpx<T>* LO, cpx<T>* LV, const spn<T>* LS, int L, int ty, int tz,
                                 int r0, int po, double hsc, double* g) {
  const int wy = ty + 4, ry = ty + 4 - 2 * r0, n = ry * (tz + 4 - 2 * r0) * L;
  for (int j = threadIdx.x; j < n; j += kTileThreads) {
    const int r = j / L, x = j - r * L;
    const int ly = r0 + r % ry, lz = r0 + r / ry;
    const int i = (lz * wy + ly) * L + x;
    const int p = (x + ly + lz) & 1;
    cpx<T>* X = (p == po) ? LO : LV;
    const cpx<T> nv = tile_advance(X, LS, i, x, L, wy * L, hsc);
    X[i] = nv;
    if (ly >= 2 && ly < ty + 2 && lz >= 2 && lz < tz + 2) {
      const double nr = nv.x, ni = nv.y;
      if (p == po) {
        g[0] += nr * nr + ni * ni;
      } else {
        const cpx<T> ap = LO[i];
        const double apr = ap.x, api = ap.y;
        g[1] += nr * nr + ni * ni;
        g[2] += apr * nr + api * ni;
        g[3] += apr * ni - api * nr;
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kTileThreads) void k_step_ov2(const Desc* __restrict__ descs,
                                                           const int* __restrict__ tileoff,
                                                           int nact, int s) {
  extern __shared__ __align__(16) unsigned char tile_smem[];
  __shared__ double red[kTileThreads / 64][8];
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  int c = 0;
  {   // the chain of this tile, from the compact table of tile offsets
    int lo = 0, hi = nact - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tileoff[mid] <= gb) lo = mid; else hi = mid - 1;
    }
    c = lo;
  }
  const Desc& D = descs[c];
  const int tl = gb - tileoff[c];
  const int L = D.L, hx = L >> 1, half = D.half, ty = D.tile_y, tz = D.tile_z;
  const int ny = L / ty, ntiles = ny * (L / tz);
  const int y0 = (tl % ny) * ty, z0 = (tl / ny) * tz;
  const int wy = ty + 4, n2 = wy * (tz + 4) * L;
  cpx<T>* LO = (cpx<T>*)tile_smem;
  cpx<T>* LV = LO + n2;
  spn<T>* LS = (spn<T>*)(LV + n2);
  const int pO = D.ctl->parity_o;
  const double hsc = -D.t / D.a;        // Ht = -(t/a) t_ij
  const bool second = s + 1 <= D.S;
  const GLOBAL spn<T>* sp = (const GLOBAL spn<T>*)D.spin;
  GLOBAL cpx<T>* vo = (GLOBAL cpx<T>*)D.vec;               // o-slots [2][half]
  GLOBAL cpx<T>* vv = (GLOBAL cpx<T>*)D.vec + D.N;         // v-slots [2][half]
  // global slot of staged site i
  auto gslot = [&](int i) -> size_t {
    const int row = i / L, x = i - row * L;
    int gy = y0 + row % wy - 2, gz = z0 + row / wy - 2;
    gy += (gy < 0) ? L : 0;
    gy -= (gy >= L) ? L : 0;
    gz += (gz < 0) ? L : 0;
    gz -= (gz >= L) ? L : 0;
    return (size_t)((x + gy + gz) & 1) * half + (x >> 1) + (size_t)hx * (gy + L * gz);
  };
  // stage: kStage sites per thread with all their loads in flight together
  constexpr int kStage = 6;
  for (int i0 = 0; i0 < n2; i0 += kStage * kTileThreads) {
    cpx<T> o[kStage], v[kStage];
    spn<T> sj[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int i = i0 + u * kTileThreads + (int)threadIdx.x;
      const size_t gs = gslot(min(i, n2 - 1));   // in bounds; the tail is not stored
      o[u] = ld(vo + gs);
      v[u] = ld(vv + gs);
      sj[u] = ld(sp + gs);
    }
    STEP_LOADS_ISSUED();
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int i = i0 + u * kTileThreads + (int)threadIdx.x;
      if (i < n2) {
        LO[i] = o[u];
        LV[i] = v[u];
        LS[i] = sj[u];
      }
    }
  }
  __syncthreads();
  double g[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // step s over the tile and one row around it (the tile alone if it is the
  // chain's last step), then step s + 1 over the tile
  tile_step(LO, LV, LS, L, ty, tz, second ? 1 : 2, pO ^ (s & 1), hsc, g);
  __syncthreads();
  if (second) {
    tile_step(LO, LV, LS, L, ty, tz, 2, pO ^ ((s + 1) & 1), hsc, g + 4);
    __syncthreads();
  }
  // write the tile's slots back
  const int n0 = ty * tz * L;
  for (int j = threadIdx.x; j < n0; j += kTileThreads) {
    const int r = j / L, x = j - r * L;
    const int i = ((2 + r / ty) * wy + 2 + r % ty) * L + x;
    const size_t gs = gslot(i);
    st(vo + gs, LO[i]);
    st(vv + gs, LV[i]);
  }
  // block sums: per wave by shuffles, then over the waves in order
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double a = g[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if (lane == 0) red[w][q] = a;
  }
  __syncthreads();
  const int nst = second ? 2 : 1;
  if (threadIdx.x < 4 * nst) {
    const int q = threadIdx.x;
    double a = 0.0;
    for (int k = 0; k < kTileThreads / 64; ++k) a += red[k][q];
    const int ss = s + (q >> 2);
    D.part[((size_t)(ss - 1) * kNP2 + (q & 3)) * D.nblk + tl] = a;
  }
  if (tl == 0) {   // partial-sum slots of this chain beyond its tiles
    const int extra = D.nblk - ntiles;
    for (int k = threadIdx.x; k < 4 * nst * extra; k += kTileThreads) {
      const int q = k / extra, b = ntiles + k % extra;
      const int ss = s + (q >> 2);
      D.part[((size_t)(ss - 1) * kNP2 + (q & 3)) * D.nblk + b] = 0.0;
    }
  }
}

// grid (Smax, n), 64 threads: pair-form moments [M][3] (oo, vv, ov):
//   mu^{oo}_{2s} = 2 P^{oo}_s - 1, mu^{vv}_{2s} = 2 P^{vv}_s - <v|v>,
//   mu^{ov}_{2s-1} = 2 Q^{ov}_s - mu^{ov}_1, mu^{ov}_1 = Q^{ov}_1; the others vanish
//   on the bipartite lattice (mu^{ov}_0 = <o|v> = 0).
__global__ __launch_bounds__(256) void k_moments_ov(const Desc* __restrict__ descs) {
  const Desc& D = descs[blockIdx.y];
  __shared__ double PP[32][6];
  const int t = threadIdx.x, col = t & 7, sl = t >> 3;
  const int s = blockIdx.x * 32 + sl + 1;
  if (s <= D.S) {
    if (col < 4) PP[sl][col] = sum_run(D.part + ((size_t)(s - 1) * kNP2 + col) * D.nblk, D.nblk);
    else if (col < 6 && s > 1) PP[sl][col] = sum_run(D.part + (size_t)(col - 2) * D.nblk, D.nblk);
  }
  __syncthreads();
  if (s > D.S || col != 0) return;
  const double* P = PP[sl];
  const Ctl* ctl = D.ctl;
  double vv0 = 0.0;   // <v|v> = sum_{de} conj(delta_d) delta_e [n_d == n_e]
  for (int d = 0; d < 6; ++d)
    for (int e = 0; e < 6; ++e)
      if (ctl->start_site[1 + d] == ctl->start_site[1 + e])
        vv0 += ctl->delta[2 * d] * ctl->delta[2 * e] + ctl->delta[2 * d + 1] * ctl->delta[2 * e + 1];
  double* mom = D.mom;
  auto put = [&](int n, int q, double re, double im) {
    mom[((size_t)n * 3 + q) * 2] = re;
    mom[((size_t)n * 3 + q) * 2 + 1] = im;
  };
  const double q1r = (s == 1) ? P[2] : P[4], q1i = (s == 1) ? P[3] : P[5];
  if (s == 1) {
    put(0, 0, 1.0, 0.0);
    put(0, 1, vv0, 0.0);
    put(0, 2, 0.0, 0.0);
  }
  put(2 * s - 1, 0, 0.0, 0.0);
  put(2 * s - 1, 1, 0.0, 0.0);
  if (s == 1) put(1, 2, q1r, q1i);
  else put(2 * s - 1, 2, 2.0 * P[2] - q1r, 2.0 * P[3] - q1i);
  if (2 * s < D.M) {
    put(2 * s, 0, 2.0 * P[0] - 1.0, 0.0);
    put(2 * s, 1, 2.0 * P[1] - vv0, 0.0);
    put(2 * s, 2, 0.0, 0.0);
  }
}

// Index of P^{de} (d <= e) in the packed 49-value block partial.
__device__ inline int pidx(int d, int e) {
  int idx = 1;
  for (int q = 0; q < d; ++q) idx += 1 + 2 * (5 - q);
  return idx + (e == d ? 0 : 1 + 2 * (e - d - 1));
}

// ------------------------------------------------------------- moments ---
// grid (ceil(Smax/4), n), 256 threads = 4 steps x 64 columns: sums the block
// partials of each step (layout [S][kNP][nblk], one contiguous run per value)
// and writes mu_{2s-1}, mu_{2s} (and mu_0 for s = 1):
//   mu_{2s}   = 2 P_s - mu_0,  mu_{2s-1} = 2 Q_s - mu_1  (s >= 2),
//   mu_1 = Q_1, mu_0^{jk} = [site_j == site_k];
// pairs that vanish on the bipartite lattice are written as exact zeros and
// the lower triangle follows from Hermiticity.
__global__ __launch_bounds__(256) void k_moments(const Desc* __restrict__ descs) {
  const Desc& D = descs[blockIdx.y];
  __shared__ double PP[4][kNP];
  __shared__ double QQ[4][12];
  const int t = threadIdx.x, col = t & 63, sl = t >> 6;
  const int s = blockIdx.x * 4 + sl + 1;
  const int nblk = D.nblk;
  if (s <= D.S) {
    if (col < kNP) {
      PP[sl][col] = sum_run(D.part + ((size_t)(s - 1) * kNP + col) * nblk, nblk);
    } else if (col < kNP + 12 && s > 1) {
      QQ[sl][col - kNP] = sum_run(D.part + ((size_t)(37 + col - kNP)) * nblk, nblk);
    }
  }
  __syncthreads();
  if (s > D.S) return;
  const double* P = PP[sl];
  const double* Q1 = QQ[sl];
  if (col >= 49) return;
  const int j = col / 7, k = col % 7;
  const Ctl* ctl = D.ctl;
  const double d0 = (ctl->start_site[j] == ctl->start_site[k]) ? 1.0 : 0.0;
  double* mom = D.mom;
  auto put = [&](int n, double re, double im) {
    mom[(((size_t)n * 7 + j) * 7 + k) * 2] = re;
    mom[(((size_t)n * 7 + j) * 7 + k) * 2 + 1] = im;
  };
  auto q1 = [&](int e, double& re, double& im) {
    if (s == 1) { re = P[37 + 2 * e]; im = P[38 + 2 * e]; }
    else { re = Q1[2 * e]; im = Q1[2 * e + 1]; }
  };
  if (s == 1) put(0, d0, 0.0);
  // odd moment n = 2s - 1
  {
    double re = 0.0, im = 0.0;
    if ((j == 0) != (k == 0)) {
      const int e = (j == 0) ? k - 1 : j - 1;
      double r1, i1;
      q1(e, r1, i1);
      if (s == 1) { re = r1; im = i1; }
      else { re = 2.0 * P[37 + 2 * e] - r1; im = 2.0 * P[38 + 2 * e] - i1; }
      if (j != 0) im = -im;   // mu^{e o} = conj(mu^{o e})
    }
    put(2 * s - 1, re, im);
  }
  // even moment n = 2s
  if (2 * s < D.M) {
    double re = 0.0, im = 0.0;
    if (j == 0 && k == 0) {
      re = 2.0 * P[0] - 1.0;
    } else if (j > 0 && k > 0) {
      const int d = (j < k ? j : k) - 1, e = (j < k ? k : j) - 1;
      const int ix = pidx(d, e);
      re = 2.0 * P[ix] - d0;
      im = (d == e) ? 0.0 : 2.0 * P[ix + 1];
      if (j > k) im = -im;
    } else {
      re = -d0;
    }
    put(2 * s, re, im);
  }
}

// -------------------------------------------------------- reconstruction ---
__device__ inline int bitrev(int v, int bits) {
  return (int)(__brev((unsigned)v) >> (32 - bits));
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Constant tables of the reconstruction of one chain (depend on M, K, the
// damping kernel, beta, mu and a only): damping g_n (Jackson, or Lorentz
// sinh(lambda(1 - n/M))/sinh(lambda)); pre-twiddles exp(-i pi m / 2K) of
// equation "mu_to_mu_tilde"; FFT twiddles exp(-2 pi i j / K); node sines
// sin th_k; quadrature weights (beta a / K) f(a w_k + b) sin th_k of
// equation "d_seff2" with w_k = cos th_k, th_k = pi (k + 1/2) / K.
__global__ void k_tables(const Desc* __restrict__ descs) {
  const Desc& D = descs[0];
  const int M = D.M, K = D.K;
  double* g = D.tab;
  double* pre = g + M;
  double* tw = pre + 2 * (size_t)K;
  double* sth = tw + (size_t)K;
  double* wt = sth + K;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) {
    if (D.kernel == GFMC_LORENTZ) {
      g[i] = sinh(D.lambda * (1.0 - (double)i / M)) / sinh(D.lambda);
    } else {
      const double qn = (double)i / (M + 1.0);
      g[i] = ((M - i + 1.0) * cospi(qn) + sinpi(qn) * cospi(1.0 / (M + 1.0)) /
                                             sinpi(1.0 / (M + 1.0))) / (M + 1.0);
    }
  }
  if (i < K) {
    double sn, cs;
    sincospi(-(double)i / (2.0 * K), &sn, &cs);
    pre[2 * i] = cs;
    pre[2 * i + 1] = sn;
    const double st = sinpi((i + 0.5) / K);
    sth[i] = st;
    const double e = D.a * cospi((i + 0.5) / K);
    const double xx = D.beta * (e - D.mu);
    double f;
    if (xx > 0) { const double qq = exp(-xx); f = qq / (1.0 + qq); }
    else f = 1.0 / (1.0 + exp(xx));
    wt[i] = D.beta * D.a / K * f * st;
  }
  if (i < K / 2) {
    double sn, cs;
    sincospi(-2.0 * i / K, &sn, &cs);
    tw[2 * i] = cs;
    tw[2 * i + 1] = sn;
  }
}

// One block per chain.  mode 0: proposal from the counter (Metropolis,
// update, counter advance); mode 1/2: evaluation only.
// Diagonal moment n of the mixed start vector q (0 |o>, 1 |v>, 2 |o>+|v>,
// 3 |o>+i|v>) from the pair moments m3 = (mu^{oo}, mu^{vv}, mu^{ov}) of
// order n: <o+v|T|o+v> = mu^{oo} + mu^{vv} + 2 Re mu^{ov},
// <o+iv|T|o+iv> = mu^{oo} + mu^{vv} - 2 Im mu^{ov}.
template <typename P>
__device__ inline double mixed_series(P m3, int q) {
  const double s = m3[0].x + m3[1].x;
  return (q == 0) ? m3[0].x : (q == 1) ? m3[1].x : (q == 2) ? s + 2.0 * m3[2].x
                                                            : s - 2.0 * m3[2].y;
}

// out[q][n] = mixed_series(mom[n], q) for one chain, n < M.
__global__ void k_mixed_series(const Desc* __restrict__ descs, double* __restrict__ out) {
  const Desc& D = descs[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * D.M) return;
  const int q = i / D.M, n = i % D.M;
  out[i] = mixed_series((const double2*)D.mom + (size_t)n * 3, q);
}

__global__ __launch_bounds__(kReconThreads) void k_recon(const Desc* __restrict__ descs,
                                                         const int32_t* __restrict__ force,
                                                         gfmc_step_record* __restrict__ recs,
                                                         int lds_items) {
  // dynamic LDS: the FFT twiddles [K/2] (when the launch reserved room for
  // them) and the transform buffer [K]
  extern __shared__ double2 dyn[];
  __shared__ double red[kReconThreads];
  __shared__ double tot[kReconThreads];
  const int c = blockIdx.x;
  const Desc& D = descs[c];
  Ctl* ctl = D.ctl;
  const int M = D.M, K = D.K, lg = D.log2K, tid = threadIdx.x;
  const double a = D.a;
  double dl[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) dl[i] = ctl->delta[i];
  // global (not flat) pointers: a flat access counts against the LDS wait
  // counter, so every LDS wait of the transforms would also wait for it
  const GLOBAL d2v* __restrict__ mom = (const GLOBAL d2v*)D.mom;   // [M][7][7]
  GLOBAL d2v* __restrict__ gs = (GLOBAL d2v*)D.gscr;               // [4][K]
  const GLOBAL double* __restrict__ gtab = (const GLOBAL double*)D.tab;   // g[M]
  const GLOBAL d2v* __restrict__ pre = (const GLOBAL d2v*)(gtab + M);
  const GLOBAL d2v* __restrict__ tw = pre + K;                     // [K/2]
  const GLOBAL double* __restrict__ sth = (const GLOBAL double*)(tw + K / 2);
  const GLOBAL double* __restrict__ wt = sth + K;
  const bool twl = K + K / 2 <= lds_items;   // twiddles staged in LDS
  double2* buf = twl ? dyn + K / 2 : dyn;
  if (twl)
    for (int i = tid; i < K / 2; i += kReconThreads) dyn[i] = make_double2(tw[i].x, tw[i].y);

  // Four real series: 0 mu^{oo}, 1 mu^{vv}, 2 Re mu^{ov}, 3 Im mu^{ov};
  // mu^{vo} = conj(mu^{ov}) (Hermitian moments), so G_vo uses the same series.
  // Mixed start vectors: 0 mu^{oo}, 1 mu^{vv}, 2 mu^{o+v}, 3 mu^{o+iv}.
  // Transform input c_m = mu'_m exp(-i pi m / (2K)) of series q (zero for m >= M).
  auto series_at = [&](int q, int m) -> double2 {
    double val = 0.0;
    if (m < M) {
      double x;
      if (D.vectors == GFMC_VECTORS_OV) {
        const GLOBAL d2v* m3 = mom + (size_t)m * 3;
        x = (q == 0) ? m3[0].x : (q == 1) ? m3[1].x : (q == 2) ? m3[2].x : m3[2].y;
      } else if (D.vectors == GFMC_VECTORS_MIXED) {
        x = mixed_series(mom + (size_t)m * 3, q);
      } else {
        const GLOBAL d2v* mm = mom + (size_t)m * 49;
        if (q == 0) {
          x = mm[0].x;
        } else if (q == 1) {
          double re = 0.0;
          for (int d = 0; d < 6; ++d) {
            double sr = 0.0, si = 0.0;   // sum_e delta_e mu^{de}
            for (int e = 0; e < 6; ++e) {
              const d2v me = mm[(1 + d) * 7 + 1 + e];
              sr += dl[2 * e] * me.x - dl[2 * e + 1] * me.y;
              si += dl[2 * e] * me.y + dl[2 * e + 1] * me.x;
            }
            re += dl[2 * d] * sr + dl[2 * d + 1] * si;   // Re(conj(delta_d) * (...))
          }
          x = re;
        } else {
          double sr = 0.0, si = 0.0;
          for (int e = 0; e < 6; ++e) {
            const d2v me = mm[1 + e];
            sr += dl[2 * e] * me.x - dl[2 * e + 1] * me.y;
            si += dl[2 * e] * me.y + dl[2 * e + 1] * me.x;
          }
          x = (q == 2) ? sr : si;
        }
      }
      val = gtab[m] * x;
      if (m == 0) val *= 0.5;
    }
    const d2v pm = pre[m];
    return make_double2(val * pm.x, val * pm.y);
  };
  // radix-2 decimation-in-time FFT stage of half-length hl over bf, butterflies
  // b0, b0 + step, ...: gamma_n = sum_m c_m exp(-2 pi i m n / K)
  auto fft_stage = [&](double2* bf, int len, int b0, int step) {
    const int hl = len >> 1;
    for (int b = b0; b < (K >> 1); b += step) {
      const int j = b % hl, base = (b / hl) * len;
      const double2 u = bf[base + j];
      const int ti = j * (K / len);
      const double2 t = cmul(bf[base + j + hl], twl ? dyn[ti] : make_double2(tw[ti].x, tw[ti].y));
      bf[base + j] = make_double2(u.x + t.x, u.y + t.y);
      bf[base + j + hl] = make_double2(u.x - t.x, u.y - t.y);
    }
  };
  // chi_{2j} = gamma_j, chi_{2j+1} = conj(gamma_{K-j-1}); Gt_k = 2i chi_k / sin th_k
  auto store_g = [&](const double2* bf, int q, int k) {
    const int j = k >> 1;
    double2 chi = bf[j];
    if (k & 1) {
      chi = bf[K - j - 1];
      chi.y = -chi.y;
    }
    const double st = sth[k];
    gs[(size_t)q * K + k] = d2v{-2.0 * chi.y / st, 2.0 * chi.x / st};
  };
  if (4 * K + K / 2 <= lds_items) {
    // room for all four transforms: one wave per series, side by side, with
    // wave-level ordering between the stages instead of block barriers
    double2* B = dyn + K / 2;   // [4][K]
    for (int idx = tid; idx < 4 * K; idx += kReconThreads) {
      const int q = idx >> lg, m = idx & (K - 1);
      B[(size_t)q * K + bitrev(m, lg)] = series_at(q, m);
    }
    __syncthreads();
    const int q = tid >> 6, lane = tid & 63;
    double2* bq = B + (size_t)q * K;
    for (int len = 2; len <= K; len <<= 1) {
      fft_stage(bq, len, lane, 64);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int k = lane; k < K; k += 64) store_g(bq, q, k);
    __syncthreads();
  } else {
    for (int q = 0; q < 4; ++q) {
      for (int m = tid; m < K; m += kReconThreads) buf[bitrev(m, lg)] = series_at(q, m);
      __syncthreads();
      for (int len = 2; len <= K; len <<= 1) {
        fft_stage(buf, len, tid, kReconThreads);
        __syncthreads();
      }
      for (int k = tid; k < K; k += kReconThreads) store_g(buf, q, k);
      __syncthreads();
    }
  }
  // d_k = (1 + G_ov)(1 + G_vo) - G_oo G_vv with G = Gt / a
  const double ia = 1.0 / a;
  for (int k = tid; k < K; k += kReconThreads) {
    const d2v g0 = gs[k], g1 = gs[(size_t)K + k], R = gs[2 * (size_t)K + k],
              I = gs[3 * (size_t)K + k];
    const double2 goo = make_double2(g0.x, g0.y), gvv = make_double2(g1.x, g1.y);
    double2 p, m;
    if (D.vectors == GFMC_VECTORS_MIXED) {
      // G_ov = [A + i (S - G_{o+iv})] / 2, G_vo = [A + i (G_{o+iv} - S)] / 2 with
      // S = G_oo + G_vv, A = G_{o+v} - S (Section 2.2, mixed diagonal elements)
      const double2 S = make_double2(goo.x + gvv.x, goo.y + gvv.y);
      const double2 A = make_double2(R.x - S.x, R.y - S.y);
      const double2 B = make_double2(I.x - S.x, I.y - S.y);   // G_{o+iv} - S
      p = make_double2(1.0 + 0.5 * ia * (A.x + B.y), 0.5 * ia * (A.y - B.x));   // 1 + G_ov
      m = make_double2(1.0 + 0.5 * ia * (A.x - B.y), 0.5 * ia * (A.y + B.x));   // 1 + G_vo
    } else {
      p = make_double2(1.0 + ia * (R.x - I.y), ia * (R.y + I.x));   // 1 + G_ov
      m = make_double2(1.0 + ia * (R.x + I.y), ia * (R.y - I.x));   // 1 + G_vo
    }
    const double2 pm = cmul(p, m);
    const double2 gg = cmul(goo, gvv);
    buf[k] = make_double2(pm.x - ia * ia * gg.x, pm.y - ia * ia * gg.y);
  }
  __syncthreads();
  // Continuous phase from the lowest node (k = K-1) upwards:
  // phi_k = Arg d_{K-1} + sum_{j=k}^{K-2} Arg(d_j conj(d_{j+1})), as a chunked suffix sum.
  const int chunk = (K + kReconThreads - 1) / kReconThreads;
  const int k0 = tid * chunk, k1 = min(K, k0 + chunk);
  auto inc = [&](int k) -> double {
    if (k == K - 1) return atan2(buf[k].y, buf[k].x);
    const double2 r = cmul(buf[k], make_double2(buf[k + 1].x, -buf[k + 1].y));
    return atan2(r.y, r.x);
  };
  double csum = 0.0;
  for (int k = k0; k < k1; ++k) csum += inc(k);
  // sum over the later chunks (an exclusive suffix sum): inclusive suffix
  // sums within each wave by shuffles, shifted by one lane, plus the totals
  // of the later waves
  const int lane = tid & 63, wv = tid >> 6;
  double x = csum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_down(x, off);
    if (lane + off < 64) x += y;
  }
  const double after = __shfl_down(x, 1);
  if (lane == 0) tot[wv] = x;
  __syncthreads();
  double later = (lane < 63) ? after : 0.0;
  for (int w2 = wv + 1; w2 < kReconThreads / 64; ++w2) later += tot[w2];
  double phi = later, part = 0.0, ptop = 0.0;
  for (int k = k1 - 1; k >= k0; --k) {
    phi += inc(k);
    part += wt[k] * phi;
    if (k == 0) ptop = phi;
  }
  red[tid] = part;
  __syncthreads();
  for (int w = kReconThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const bool failed = ctl->bar[3] != 0u;   // the persistent step run timed out
    const double ds = failed ? __builtin_nan("") : red[0];
    ctl->dseff = ds;
    ctl->phase_top = ptop;
    if (ctl->mode == 0 && !failed) {
      // a non-finite Delta S (corrupted chain state) is rejected whatever the
      // forcing, and counted, so that the chain is flagged and left unchanged
      const bool finite = isfinite(ds);
      const double u = ctl->u;
      const int own = (finite && (ds <= 0.0 || u < exp(-ds))) ? 1 : 0;
      const int f = force ? force[c] : -1;
      const int acc = !finite ? 0 : (f < 0 ? own : (f ? 1 : 0));
      if (!finite) ctl->nonfinite += 1;
      const int o = ctl->site;
      if (recs) {
        gfmc_step_record& R = recs[c];
        R.index = ctl->index; R.site = o; R.own = own; R.accepted = acc; R.pad_ = 0;
        R.theta_old = ctl->th_old; R.phi_old = ctl->ph_old;
        R.theta_new = ctl->th_new; R.phi_new = ctl->ph_new;
        R.dseff = ds; R.u = u; R.phase_top = ptop;
      }
      ctl->own = own;
      ctl->accepted = acc;
      if (acc) {
        D.theta[o] = ctl->th_new;
        D.phi[o] = ctl->ph_new;
      }
      ctl->index += 1;
      ctl->accepted_total += acc;
    }
  }
}

// Spinor cache update for an accepted move (separate so that it runs in the
// recursion precision).
// Stored hopping row of `site`: t_{site, n_d(site)} = <chi_site|chi_{n_d}> from
// the spinor cache (the same arithmetic as the recomputing step kernel).
template <typename T>
__device__ inline void build_row(const Desc& D, int site) {
  int x, y, z;
  site_xyz(site, D.L, x, y, z);
  const int par = (x + y + z) & 1, hh = half_index(x, y, z, D.L);
  const spn<T>* sp = (const spn<T>*)D.spin;
  const spn<T> si = sp[(size_t)par * D.half + hh];
  six<T> row;
  for (int d = 0; d < 6; ++d) {
    const int nh = nb_half(x, y, z, d, D.L);
    const spn<T> sj = sp[(size_t)(par ^ 1) * D.half + nh];
    hop_spinor(si, sj, -D.t / D.a, row.v[d].x, row.v[d].y);
  }
  planes<T>(D.hop, D.N).st((size_t)par * D.half + hh, row);
}

template <typename T>
__global__ void k_hops(const Desc* __restrict__ descs) {
  const Desc& D = descs[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D.N && D.hop) build_row<T>(D, i);
}

template <typename T>
__global__ void k_accept_spinor(const Desc* __restrict__ descs, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const Desc& D = descs[c];
  const Ctl* ctl = D.ctl;
  if (ctl->mode != 0 || !ctl->accepted) return;
  spn<T>* sp = (spn<T>*)D.spin;
  sp[(size_t)ctl->parity_o * D.half + ctl->o_half] = make_spinor<T>(ctl->th_new, ctl->ph_new);
  if (D.hop)   // rows of o and of its neighbours change
    for (int j = 0; j < 7; ++j) build_row<T>(D, ctl->start_site[j]);
}

// ---------------------------------------------------------- per-site ops ---
template <typename T>
__global__ void k_spinors(const Desc* __restrict__ descs) {
  const Desc& D = descs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  int x, y, z;
  site_xyz(i, D.L, x, y, z);
  spn<T>* sp = (spn<T>*)D.spin;
  sp[(size_t)((x + y + z) & 1) * D.half + half_index(x, y, z, D.L)] =
      make_spinor<T>(D.theta[i], D.phi[i]);
}

// Initial spins: mode 0 uniform on the sphere from counter (i, 2, 0, 0);
// modes 1, 2 ferromagnetic (the random subset of mode 2 follows in k_fisher_yates).
__global__ void k_init_spins(const Desc* __restrict__ descs, int mode) {
  const Desc& D = descs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  if (mode == 0) {
    uint64_t r[4];
    philox((uint64_t)i, 2ULL, D.seed, D.chain_id, r);
    D.theta[i] = acos(1.0 - 2.0 * u01(r[0]));
    D.phi[i] = 2.0 * M_PI * u01(r[1]);
  } else {
    D.theta[i] = 0.0;
    D.phi[i] = 0.0;
  }
}

// Exactly nr distinct sites by a partial Fisher-Yates shuffle (pick k from
// counter (k, 3, 0, 0)), each redrawn on the sphere from (site, 2, 0, 0).
// Sequential by construction; `perm` is N int32 of scratch.
__global__ void k_fisher_yates(const Desc* __restrict__ descs, int64_t nr, int32_t* perm) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const Desc& D = descs[0];
  const int64_t N = D.N;
  for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
  for (int64_t k = 0; k < nr; ++k) {
    uint64_t r[4];
    philox((uint64_t)k, 3ULL, D.seed, D.chain_id, r);
    const int64_t j = k + (int64_t)__umul64hi(r[0], (uint64_t)(N - k));
    const int32_t tmp = perm[k];
    perm[k] = perm[j];
    perm[j] = tmp;
  }
  for (int64_t k = 0; k < nr; ++k) {
    const int i = perm[k];
    uint64_t r[4];
    philox((uint64_t)i, 2ULL, D.seed, D.chain_id, r);
    D.theta[i] = acos(1.0 - 2.0 * u01(r[0]));
    D.phi[i] = 2.0 * M_PI * u01(r[1]);
  }
}

// |sum_i S_i| / N, one block per chain, written to out[c].
__global__ void k_magnetization(const Desc* __restrict__ descs, double* __restrict__ out) {
  __shared__ double rs[3][256];
  const Desc& D = descs[blockIdx.x];
  double sx = 0, sy = 0, sz = 0;
  for (int i = threadIdx.x; i < D.N; i += blockDim.x) {
    double st, ct, sp, cp;
    sincos(D.theta[i], &st, &ct);
    sincos(D.phi[i], &sp, &cp);
    sx += st * cp;
    sy += st * sp;
    sz += ct;
  }
  rs[0][threadIdx.x] = sx;
  rs[1][threadIdx.x] = sy;
  rs[2][threadIdx.x] = sz;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) rs[q][threadIdx.x] += rs[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    out[blockIdx.x] = sqrt(rs[0][0] * rs[0][0] + rs[1][0] * rs[1][0] + rs[2][0] * rs[2][0]) / D.N;
}

// ------------------------------------------------------------ launchers ---
hipError_t launch_mixed_series(const Desc* d, int M, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mixed_series, dim3((4 * M + 255) / 256), dim3(256), 0, st, d, out);
  return hipGetLastError();
}

hipError_t launch_propose(const Desc* d, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_propose, dim3(n), dim3(64), 0, st, d, n);
  return hipGetLastError();
}

template <typename T, int PPT, bool HOPS, int BT>
hipError_t launch_step_t(int ov, int nt, const Desc* d, const int* blkoff, int nact, int blocks,
                         int s, const int* act_end, hipStream_t st) {
  const dim3 g(blocks), b(BT);
  // round launches (act_end) never run step 1: it has a launch of its own
  const bool first = !act_end && s == 1;
  if (ov) {
    if constexpr (BT != kStepThreads) {
      return hipErrorInvalidValue;   // the pair kernels run 256-thread blocks only
    } else if (first) {
      hipLaunchKernelGGL((k_step_ov<T, true, PPT>), g, b, 0, st, d, blkoff, nact, s, act_end);
    } else {
      hipLaunchKernelGGL((k_step_ov<T, false, PPT>), g, b, 0, st, d, blkoff, nact, s, act_end);
    }
  } else if (first) {
    hipLaunchKernelGGL((k_step<T, true, PPT, HOPS, false, BT>), g, b, 0, st, d, blkoff, nact, s,
                       act_end);
  } else if (nt) {
    hipLaunchKernelGGL((k_step<T, false, PPT, HOPS, true, BT>), g, b, 0, st, d, blkoff, nact, s,
                       act_end);
  } else {
    hipLaunchKernelGGL((k_step<T, false, PPT, HOPS, false, BT>), g, b, 0, st, d, blkoff, nact, s,
                       act_end);
  }
  return hipGetLastError();
}

template <typename T, bool HOPS, int BT>
hipError_t launch_step_h(int ov, int nt, int ppt, const Desc* d, const int* blkoff, int nact,
                         int blocks, int s, const int* act_end, hipStream_t st) {
  return ppt == 2 ? launch_step_t<T, 2, HOPS, BT>(ov, nt, d, blkoff, nact, blocks, s, act_end, st)
                  : launch_step_t<T, 1, HOPS, BT>(ov, nt, d, blkoff, nact, blocks, s, act_end, st);
}

// bt: threads per block, 256 or (7-vector form, hoppings recomputed) 512
hipError_t launch_step(int fp32, int ov, int hops, int ppt, const Desc* d, const int* blkoff,
                       int nact, int blocks, int s, hipStream_t st, const int* act_end, int nt,
                       int bt) {
  if (bt == 512) {
    if (ov || hops) return hipErrorInvalidValue;
    return fp32 ? launch_step_h<float, false, 512>(0, nt, ppt, d, blkoff, nact, blocks, s,
                                                   act_end, st)
                : launch_step_h<double, false, 512>(0, nt, ppt, d, blkoff, nact, blocks, s,
                                                    act_end, st);
  }
  if (bt != kStepThreads) return hipErrorInvalidValue;
  if (fp32)
    return hops ? launch_step_h<float, true, kStepThreads>(ov, nt, ppt, d, blkoff, nact, blocks,
                                                           s, act_end, st)
                : launch_step_h<float, false, kStepThreads>(ov, nt, ppt, d, blkoff, nact, blocks,
                                                            s, act_end, st);
  return hops ? launch_step_h<double, true, kStepThreads>(ov, nt, ppt, d, blkoff, nact, blocks, s,
                                                          act_end, st)
              : launch_step_h<double, false, kStepThreads>(ov, nt, ppt, d, blkoff, nact, blocks,
                                                           s, act_end, st);
}

// The two-step pair kernel takes up to kTileLds of dynamic LDS (set once per
// process, before its first launch).
hipError_t prepare_step_ov2() {
  static const hipError_t e = [] {
    hipError_t r = hipFuncSetAttribute((const void*)k_step_ov2<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kTileLds);
    if (r == hipSuccess)
      r = hipFuncSetAttribute((const void*)k_step_ov2<double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kTileLds);
    return r;
  }();
  return e;
}

hipError_t launch_step_ov2(int fp32, const Desc* d, const int* tileoff, int nact, int tiles, int s,
                           size_t lds, hipStream_t st) {
  const hipError_t e = prepare_step_ov2();
  if (e != hipSuccess) return e;
  if (fp32)
    hipLaunchKernelGGL(k_step_ov2<float>, dim3(tiles), dim3(kTileThreads), lds, st, d, tileoff,
                       nact, s);
  else
    hipLaunchKernelGGL(k_step_ov2<double>, dim3(tiles), dim3(kTileThreads), lds, st, d, tileoff,
                       nact, s);
  return hipGetLastError();
}

hipError_t launch_hops(int fp32, const Desc* d, int nmax, hipStream_t st) {
  if (fp32) hipLaunchKernelGGL(k_hops<float>, dim3((nmax + 255) / 256), dim3(256), 0, st, d);
  else hipLaunchKernelGGL(k_hops<double>, dim3((nmax + 255) / 256), dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_moments(int ov, const Desc* d, int n, int smax, hipStream_t st) {
  if (ov) hipLaunchKernelGGL(k_moments_ov, dim3((smax + 31) / 32, n), dim3(256), 0, st, d);
  else hipLaunchKernelGGL(k_moments, dim3((smax + 3) / 4, n), dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_recon(int fp32, const Desc* d, int n, int kmax, const int32_t* force,
                        gfmc_step_record* recs, hipStream_t st) {
  static const bool attr_done = [] {   // thread-safe one-time setup
    return hipFuncSetAttribute((const void*)k_recon, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (kMaxK + kMaxK / 8) * (int)sizeof(double2)) == hipSuccess;
  }();
  (void)attr_done;
  // dynamic LDS in 16-byte items: the twiddles and four transform buffers
  // side by side up to K = 2048, the twiddles and one buffer up to 4096,
  // else one buffer
  const int items = (kmax <= kMaxK / 4) ? 4 * kmax + kmax / 2
                    : (kmax <= kMaxK / 2) ? kmax + kmax / 2 : kmax;
  hipLaunchKernelGGL(k_recon, dim3(n), dim3(kReconThreads), (size_t)items * sizeof(double2), st,
                     d, force, recs, items);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (fp32)
    hipLaunchKernelGGL(k_accept_spinor<float>, dim3((n + 63) / 64), dim3(64), 0, st, d, n);
  else
    hipLaunchKernelGGL(k_accept_spinor<double>, dim3((n + 63) / 64), dim3(64), 0, st, d, n);
  return hipGetLastError();
}

hipError_t launch_spinors(int fp32, const Desc* d, int n, int nmax, hipStream_t st) {
  dim3 g((nmax + 255) / 256, n);
  if (fp32) hipLaunchKernelGGL(k_spinors<float>, g, dim3(256), 0, st, d);
  else hipLaunchKernelGGL(k_spinors<double>, g, dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_init_spins(const Desc* d, int nmax, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_init_spins, dim3((nmax + 255) / 256, 1), dim3(256), 0, st, d, mode);
  return hipGetLastError();
}

hipError_t launch_fisher_yates(const Desc* d, int64_t nr, int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL(k_fisher_yates, dim3(1), dim3(1), 0, st, d, nr, perm);
  return hipGetLastError();
}

template <int BT>
hipError_t launch_persist_t(int fp32, const Desc* d, int nb, hipStream_t st) {
  // eight blocks per working block: nb of them land on every die
  void* args[] = {(void*)&d, (void*)&nb};
  const dim3 g(8 * nb), b(BT);
  if (fp32)
    return hipLaunchCooperativeKernel((const void*)k_persist<float, BT>, g, b, args, 0, st);
  return hipLaunchCooperativeKernel((const void*)k_persist<double, BT>, g, b, args, 0, st);
}

hipError_t launch_persist(int fp32, const Desc* d, int nb, int threads, hipStream_t st) {
  if (threads == 64) return launch_persist_t<64>(fp32, d, nb, st);
  if (threads == 128) return launch_persist_t<128>(fp32, d, nb, st);
  if (threads == 256) return launch_persist_t<256>(fp32, d, nb, st);
  return hipErrorInvalidValue;
}

hipError_t launch_die_census(unsigned* counts, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_die_census, dim3(blocks), dim3(64), 0, st, counts);
  return hipGetLastError();
}

hipError_t launch_magnetization(const Desc* d, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_magnetization, dim3(n), dim3(256), 0, st, d, out);
  return hipGetLastError();
}

}  // namespace gfmc

namespace gfmc {
hipError_t launch_tables(const Desc* d, int kmax, hipStream_t st) {
  hipLaunchKernelGGL(k_tables, dim3((kmax + 255) / 256), dim3(256), 0, st, d);
  return hipGetLastError();
}
}  // namespace gfmc

namespace gfmc {
hipError_t launch_resident(int fp32, const Desc* d, int n, size_t lds, hipStream_t st) {
  static const bool attr_done = [] {   // thread-safe one-time setup
    return hipFuncSetAttribute((const void*)k_resident<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, kResidentLds) ==
               hipSuccess &&
           hipFuncSetAttribute((const void*)k_resident<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, kResidentLds) ==
               hipSuccess;
  }();
  (void)attr_done;
  if (fp32) hipLaunchKernelGGL(k_resident<float>, dim3(n), dim3(kResThreads), lds, st, d);
  else hipLaunchKernelGGL(k_resident<double>, dim3(n), dim3(kResThreads), lds, st, d);
  return hipGetLastError();
}
}  // namespace gfmc
