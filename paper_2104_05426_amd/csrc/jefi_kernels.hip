// gfx950 kernels for the discretised Jefimenko sums.
//
// Built with -ffp-contract=off: every FMA in this file is written out
// explicitly, so the canonical FP64 slice-index sequence (coordinates as
// origin + index*spacing, R = sqrt((dx*dx + dy*dy) + dz*dz), u = a_f - R/(c dt))
// is evaluated exactly as specified.
//
// Pair kernel design (one workgroup = one 8x8x8 observation tile x one range
// of source bricks):
//   * each lane owns one observation point; a wavefront covers a compact
//     4x4x4 block so neighbouring lanes read neighbouring history slices;
//   * source cells come in 2x2x2 bricks; per round a workgroup computes, for
//     G bricks, the window of slices [wlo, whi] its tile can reach (from the
//     FP64 min/max tile-brick distances), skips bricks whose whole window is
//     before the oldest slice, and stages the window into LDS as four planes
//     h_k, S_k = h_(k+1) - h_k, D_k = (h_k - h_(k-1))/dt and T_k = D_(k+1) - D_k
//     so that value and backward difference at the retarded time are one FMA
//     each: v = h_k + f S_k, v_dot = D_k + f T_k;
//   * the FP32 path computes R with rsqrt and the slice index in FP32; when
//     the fractional position lies within the proven error band of a slice
//     boundary it recomputes the canonical FP64 sequence, so the index is
//     identical to the FP64 decision;
//   * screening is tested per pair (canonical FP64) only in bricks whose box
//     comes within the screening width of the tile box;
//   * FP32 block sums over two staging rounds (the fast pair kernels) or one
//     (the chunked kernel) feed compensated (two-sum) FP32 running totals;
//     the per-point totals are reduced in FP64 across splits by the epilogue
//     in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>

#include "jefi_internal.h"

namespace jefi {
namespace {

__device__ __forceinline__ double canon(double o, int i, double h) { return o + (double)i * h; }

// Canonical FP64 position of the retarded time in slice units relative to
// a_i, from the canonical separation d.
__device__ __forceinline__ double canon_u(double dx, double dy, double dz, double af, double icdt) {
  double r2 = (dx * dx + dy * dy) + dz * dz;
  double R = __builtin_sqrt(r2);
  return af - R * icdt;
}

template <class S3>
__device__ __forceinline__ bool canon_screened(double dx, double dy, double dz, const S3& s) {
  if (__builtin_fabs(dx) <= s[0] && __builtin_fabs(dy) <= s[1] && __builtin_fabs(dz) <= s[2])
    return true;
  double r2 = (dx * dx + dy * dy) + dz * dz;
  return __builtin_sqrt(r2) == 0.0;
}

// Largest FP64 r2 >= 0 whose canonical retarded position a_f - sqrt(r2)/(c dt)
// is >= N (-1 when even r2 = 0 falls short): a bisection over the ordered
// bit patterns of the non-negative doubles, with the same correctly rounded
// sqrt, multiply and subtract as the canonical sequence.
__device__ __forceinline__ double r2_threshold(int N, double af, double icdt) {
  const double n = (double)N;
  if (!(af - __builtin_sqrt(0.0) * icdt >= n)) return -1.0;
  unsigned long long lo = 0ull, hi = 0x7ff0000000000000ull;
  while (hi - lo > 1ull) {
    const unsigned long long mid = lo + ((hi - lo) >> 1);
    const double x = __longlong_as_double((long long)mid);
    if (af - __builtin_sqrt(x) * icdt >= n)
      lo = mid;
    else
      hi = mid;
  }
  return __longlong_as_double((long long)lo);
}

// Logical workgroup (split * n_tiles + tile) of hardware workgroup `bid`.
// The hardware deals workgroups round-robin over the 8 XCDs (each with its
// own L2).  With a multiple of 8 splits, XCD x takes splits x, x+8, x+16,
// ..., each with all its tiles in a row: the workgroups one XCD runs at a
// time read the source bricks of one split, and every XCD gets splits from
// all over the source, so their shares of live pairs match (contiguous
// splits would hand one XCD the edge of the source and another its
// middle).  Otherwise consecutive logical ids stay on one XCD.
__device__ __forceinline__ int xcd_remap(int bid, int n, int n_tiles, int n_splits) {
  const int x = bid & 7, l = bid >> 3;
  if ((n_splits & 7) == 0) {
    const int k = l / n_tiles;
    return (x + 8 * k) * n_tiles + (l - k * n_tiles);
  }
  const int q = n >> 3, r = n & 7;
  return x * q + min(x, r) + l;
}

// FP32 slice decision with the FP64 fallback near slice boundaries.
// Returns floor(u) (clamped below at -1e9) and the weight f.
// FP32 squared separation, x^2 + (y^2 + z^2) without contraction; the fast
// pair path forms the same expression from per-brick partial squares.
// floor(x + 0.5) as an integer in one instruction (|x| well inside int range).
__device__ __forceinline__ int cvt_nearest(float x) {
  int n;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(n) : "v"(x));
  return n;
}

__device__ __forceinline__ float r2_f32(float dx, float dy, float dz) {
  return dx * dx + (dy * dy + dz * dz);
}

template <class Canon>
__device__ __forceinline__ void index_f32(float dx, float dy, float dz, float af, float halfg,
                                          Canon canon_fn, float& m, float& f, float& ri) {
  // separations in units of c dt: R = r2 * rsq(r2) is then in slice units
  float r2 = r2_f32(dx, dy, dz);
  ri = __builtin_amdgcn_rsqf(r2);
  float u = __builtin_fmaf(-r2, ri, af);
  float fl = __builtin_floorf(u);
  float fr = u - fl;
  // NaN (a separation below FP32 resolution) also takes the FP64 decision
  if (__builtin_expect(!(__builtin_fabsf(fr - 0.5f) <= halfg), 0)) {
    double u64 = canon_fn();
    double m64 = __builtin_floor(u64);
    fl = (float)__builtin_fmax(m64, -1e9);
    fr = (float)(u64 - m64);
  }
  m = __builtin_fmaxf(fl, -1e9f);
  f = fr;
}

template <typename T>
struct Traits;
template <>
struct Traits<float> {
  static constexpr int kPlanes = 4;  // h, S, D, T; each float4 (rho, Jx, Jy, Jz)
};
template <>
struct Traits<double> {
  static constexpr int kPlanes = 8;  // (h.rho,h.Jx),(h.Jy,h.Jz),(S..),(S..),(D..),(D..),(T..),(T..)
};

__device__ __forceinline__ void two_sum_acc(float& s, float& c, float x) {
  float t = s + x;
  float bp = t - s;
  float e = (s - (t - bp)) + (x - bp);
  s = t;
  c += e;
}

// Four channels of one cell at logical slice j: zero after slice nt-1, and
// before slice 0 zero or (held past) slice 0's values.
template <class PP>
__device__ __forceinline__ float4 ring4(const float* ring, const PP& p, int j, int b, int c) {
  if (j < 0 && (p.stencil & (kStencilHold | kStencilCut))) j = 0;  // slice 0 extends backwards
  if (j < 0 || j > p.nt - 1) return make_float4(0.f, 0.f, 0.f, 0.f);
  int slot = p.slot_base + j;
  if (slot >= p.capacity) slot -= p.capacity;
  return *(const float4*)(ring + (long long)slot * p.slot_elems + ((long long)b * kBrickCells + c) * 4);
}

template <class PP>
__device__ __forceinline__ void ring4(const double* ring, const PP& p, int j, int b, int c,
                                      double out[4]) {
  if (j < 0 && (p.stencil & (kStencilHold | kStencilCut))) j = 0;
  if (j < 0 || j > p.nt - 1) {
    out[0] = out[1] = out[2] = out[3] = 0.0;
    return;
  }
  int slot = p.slot_base + j;
  if (slot >= p.capacity) slot -= p.capacity;
  const double2* q =
      (const double2*)(ring + (long long)slot * p.slot_elems + ((long long)b * kBrickCells + c) * 4);
  const double2 lo = q[0], hi = q[1];
  out[0] = lo.x; out[1] = lo.y; out[2] = hi.x; out[3] = hi.y;
}

// ---- staging helpers: raw slices to (h, S, D, T) entries ----

struct D4 {
  double x, y, z, w;
};

template <class PP>
__device__ __forceinline__ void load_raw(const float* ring, const PP& p, int jj, int b, int c,
                                         float4& out) {
  out = ring4(ring, p, jj, b, c);
}

template <class PP>
__device__ __forceinline__ void load_raw(const double* ring, const PP& p, int jj, int b, int c,
                                         D4& out) {
  double v[4];
  ring4(ring, p, jj, b, c, v);
  out = D4{v[0], v[1], v[2], v[3]};
}

// Raw buffer resource word 3 for gfx9-family targets (32-bit data, no
// swizzle); offsets at or beyond the resource's byte count read as zero.
constexpr int kRawBufferFlags = 0x00020000;
constexpr int kOutOfRange = 0x7ffffff0;  // above any ring the buffer path takes
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void buffer_raw(__amdgpu_buffer_rsrc_t rs, int off, float4& out) {
  const f32x4_t v = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  out = make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void buffer_raw(__amdgpu_buffer_rsrc_t rs, int off, D4& out) {
  const f64x2_t lo = __builtin_bit_cast(f64x2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  const f64x2_t hi = __builtin_bit_cast(f64x2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 16, 0));
  out = D4{lo.x, lo.y, hi.x, hi.y};
}

// The same loads with a wavefront-uniform part of the offset in soff (a
// scalar register) and the per-lane part in voff.
__device__ __forceinline__ void buffer_raw(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, float4& out) {
  const f32x4_t v = __builtin_bit_cast(f32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  out = make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void buffer_raw(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, D4& out) {
  const f64x2_t lo = __builtin_bit_cast(f64x2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  const f64x2_t hi = __builtin_bit_cast(f64x2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16u, soff, 0));
  out = D4{lo.x, lo.y, hi.x, hi.y};
}


template <typename T>
struct RawOf;
template <>
struct RawOf<float> {
  using type = float4;
};
template <>
struct RawOf<double> {
  using type = D4;
};

// Entry (h, S, D, T) of slot k from raw slices k-1, k, k+1, written to the
// planes: value h_k + f S, derivative D + f T.  Backward differences (the
// default): D = (h_k - h_(k-1))/dt, T = D_(k+1) - D_k.  Slope of the
// interpolant (SLOPE): D = (h_(k+1) - h_k)/dt, T = 0.
template <bool SLOPE>
__device__ __forceinline__ void put_entry(float4* lds, int PU, int idx, const float4& hm, const float4& h0,
                                          const float4& h1, float inv_dt, bool value = true) {
  float4 S, D, Tn;
  S.x = h1.x - h0.x; S.y = h1.y - h0.y; S.z = h1.z - h0.z; S.w = h1.w - h0.w;
  if (SLOPE) {
    D.x = S.x * inv_dt; D.y = S.y * inv_dt; D.z = S.z * inv_dt; D.w = S.w * inv_dt;
    Tn = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    D.x = (h0.x - hm.x) * inv_dt; D.y = (h0.y - hm.y) * inv_dt;
    D.z = (h0.z - hm.z) * inv_dt; D.w = (h0.w - hm.w) * inv_dt;
    Tn.x = S.x * inv_dt - D.x; Tn.y = S.y * inv_dt - D.y;
    Tn.z = S.z * inv_dt - D.z; Tn.w = S.w * inv_dt - D.w;
  }
  lds[idx] = value ? h0 : make_float4(0.f, 0.f, 0.f, 0.f);
  lds[PU + idx] = S;
  lds[2 * PU + idx] = D;
  lds[3 * PU + idx] = Tn;
}

template <bool SLOPE>
__device__ __forceinline__ void put_entry(float4* lds, int PU, int idx, const D4& hm, const D4& h0,
                                          const D4& h1, double inv_dt, bool value = true) {
  const double a[4] = {hm.x, hm.y, hm.z, hm.w};
  const double b[4] = {h0.x, h0.y, h0.z, h0.w};
  const double c[4] = {h1.x, h1.y, h1.z, h1.w};
  double S[4], D[4], Tn[4];
  for (int q = 0; q < 4; ++q) {
    S[q] = c[q] - b[q];
    if (SLOPE) {
      D[q] = S[q] * inv_dt;
      Tn[q] = 0.0;
    } else {
      D[q] = (b[q] - a[q]) * inv_dt;
      Tn[q] = S[q] * inv_dt - D[q];
    }
  }
  double2* l2 = (double2*)lds;
  l2[idx] = value ? make_double2(b[0], b[1]) : make_double2(0.0, 0.0);
  l2[PU + idx] = value ? make_double2(b[2], b[3]) : make_double2(0.0, 0.0);
  l2[2 * PU + idx] = make_double2(S[0], S[1]);
  l2[3 * PU + idx] = make_double2(S[2], S[3]);
  l2[4 * PU + idx] = make_double2(D[0], D[1]);
  l2[5 * PU + idx] = make_double2(D[2], D[3]);
  l2[6 * PU + idx] = make_double2(Tn[0], Tn[1]);
  l2[7 * PU + idx] = make_double2(Tn[2], Tn[3]);
}

// Entry of slot k for cubic time interpolation: the coefficients c0 .. c3 in
// f of the cubic through raw slices k-2, k-1, k, k+1 (nodes -2 .. 1), taken
// from differences to h_k so that equal slices give exactly zero higher
// coefficients; value c0 + c1 f + c2 f^2 + c3 f^3, derivative in f
// c1 + 2 c2 f + 3 c3 f^2 (scaled to time by the pair loop).
__device__ __forceinline__ void cubic_coef(float h2, float h1, float h0, float hp, float c[4]) {
  const float a = h2 - h0, b = h1 - h0, q = hp - h0;
  c[0] = h0;
  c[1] = __builtin_fmaf(a, 1.f / 6.f, __builtin_fmaf(q, 1.f / 3.f, -b));
  c[2] = (b + q) * 0.5f;
  c[3] = __builtin_fmaf(q - a, 1.f / 6.f, b * 0.5f);
}

__device__ __forceinline__ void cubic_coef(double h2, double h1, double h0, double hp, double c[4]) {
  const double a = h2 - h0, b = h1 - h0, q = hp - h0;
  c[0] = h0;
  c[1] = __builtin_fma(a, 1.0 / 6.0, __builtin_fma(q, 1.0 / 3.0, -b));
  c[2] = (b + q) * 0.5;
  c[3] = __builtin_fma(q - a, 1.0 / 6.0, b * 0.5);
}

__device__ __forceinline__ void put_cubic(float4* lds, int PU, int idx, const float4& h2, const float4& h1,
                                          const float4& h0, const float4& hp, bool value = true) {
  float cx[4], cy[4], cz[4], cw[4];
  cubic_coef(h2.x, h1.x, h0.x, hp.x, cx);
  cubic_coef(h2.y, h1.y, h0.y, hp.y, cy);
  cubic_coef(h2.z, h1.z, h0.z, hp.z, cz);
  cubic_coef(h2.w, h1.w, h0.w, hp.w, cw);
  if (!value) cx[0] = cy[0] = cz[0] = cw[0] = 0.f;
  for (int i = 0; i < 4; ++i) lds[i * PU + idx] = make_float4(cx[i], cy[i], cz[i], cw[i]);
}

__device__ __forceinline__ void put_cubic(float4* lds, int PU, int idx, const D4& h2, const D4& h1, const D4& h0,
                                          const D4& hp, bool value = true) {
  double cx[4], cy[4], cz[4], cw[4];
  cubic_coef(h2.x, h1.x, h0.x, hp.x, cx);
  cubic_coef(h2.y, h1.y, h0.y, hp.y, cy);
  cubic_coef(h2.z, h1.z, h0.z, hp.z, cz);
  cubic_coef(h2.w, h1.w, h0.w, hp.w, cw);
  if (!value) cx[0] = cy[0] = cz[0] = cw[0] = 0.0;
  double2* l2 = (double2*)lds;
  for (int i = 0; i < 4; ++i) {
    l2[2 * i * PU + idx] = make_double2(cx[i], cy[i]);
    l2[(2 * i + 1) * PU + idx] = make_double2(cz[i], cw[i]);
  }
}


// Source values (rho, Jx, Jy, Jz) and their time derivatives at fraction f
// of LDS entry e.  Linear planes (h, S, D, T): value h + f S, derivative
// D + f T (the derivative planes carry the time unit).  Cubic planes
// (c0 .. c3): value and derivative in one Horner pass, the derivative in f
// times dsc (1/dt; c in the FP32 kernels, which measure time in steps and
// lengths in c dt).
template <bool CUB>
__device__ __forceinline__ void entry_at(const float4* lds, int PU, int e, float f, float dsc, float v[4],
                                         float w[4]) {
  const float4 a4 = lds[e], b4 = lds[PU + e], c4 = lds[2 * PU + e], d4 = lds[3 * PU + e];
  const float A[4] = {a4.x, a4.y, a4.z, a4.w}, Bq[4] = {b4.x, b4.y, b4.z, b4.w};
  const float Cq[4] = {c4.x, c4.y, c4.z, c4.w}, Dq[4] = {d4.x, d4.y, d4.z, d4.w};
  if constexpr (!CUB) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = __builtin_fmaf(f, Bq[q], A[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = __builtin_fmaf(f, Dq[q], Cq[q]);
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    {
      const float p1 = __builtin_fmaf(Dq[q], f, Cq[q]);
      const float d1 = __builtin_fmaf(Dq[q], f, p1);
      const float p2 = __builtin_fmaf(p1, f, Bq[q]);
      const float d2 = __builtin_fmaf(d1, f, p2);
      v[q] = __builtin_fmaf(p2, f, A[q]);
      w[q] = d2 * dsc;
    }
  }
}

// FP64 entries: the eight 16-byte plane reads of entry e, then the value
// and derivative at fraction f from them (as for FP32).
__device__ __forceinline__ void planes_at(const float4* lds, int PU, int e, double P[4][4]) {
  const double2* l2 = (const double2*)lds;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 lo = l2[2 * i * PU + e], hi = l2[(2 * i + 1) * PU + e];
    P[i][0] = lo.x; P[i][1] = lo.y; P[i][2] = hi.x; P[i][3] = hi.y;
  }
}

template <bool CUB>
__device__ __forceinline__ void entry_from(const double P[4][4], double f, double dsc, double v[4], double w[4]) {
  if constexpr (!CUB) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = __builtin_fma(f, P[1][q], P[0][q]);
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = __builtin_fma(f, P[3][q], P[2][q]);
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    {
      const double p1 = __builtin_fma(P[3][q], f, P[2][q]);
      const double d1 = __builtin_fma(P[3][q], f, p1);
      const double p2 = __builtin_fma(p1, f, P[1][q]);
      const double d2 = __builtin_fma(d1, f, p2);
      v[q] = __builtin_fma(p2, f, P[0][q]);
      w[q] = d2 * dsc;
    }
  }
}

template <bool CUB>
__device__ __forceinline__ void entry_at(const float4* lds, int PU, int e, double f, double dsc, double v[4],
                                         double w[4]) {
  double P[4][4];
  planes_at(lds, PU, e, P);
  entry_from<CUB>(P, f, dsc, v, w);
}

// Geometry of one observation tile: first/last point indices, the FP64
// reference point (first point) and the far corner of its box.
struct TileGeom {
  int ix0, iy0, iz0, ix1, iy1, iz1;
  double refx, refy, refz, thix, thiy, thiz;
};

template <class PP>
__device__ __forceinline__ TileGeom tile_geom(const PP& p, int tile) {
  TileGeom g;
  const int tx = tile % p.ntx;
  const int ty = (tile / p.ntx) % p.nty;
  const int tz = tile / (p.ntx * p.nty);
  g.ix0 = tx * kTileEdge;
  g.iy0 = ty * kTileEdge;
  g.iz0 = tz * p.tile_z;
  g.ix1 = min(g.ix0 + kTileEdge - 1, p.obs.n[0] - 1);
  g.iy1 = min(g.iy0 + kTileEdge - 1, p.obs.n[1] - 1);
  g.iz1 = min(g.iz0 + p.tile_z - 1, p.obs.n[2] - 1);
  g.refx = canon(p.obs.o[0], g.ix0, p.obs.h[0]);
  g.refy = canon(p.obs.o[1], g.iy0, p.obs.h[1]);
  g.refz = canon(p.obs.o[2], g.iz0, p.obs.h[2]);
  g.thix = canon(p.obs.o[0], g.ix1, p.obs.h[0]);
  g.thiy = canon(p.obs.o[1], g.iy1, p.obs.h[1]);
  g.thiz = canon(p.obs.o[2], g.iz1, p.obs.h[2]);
  return g;
}

// Window of slices brick b can need for the tile: FP64 min/max separations
// of the two boxes of cell centres bound every pair's slice index (FP
// subtraction, squaring, sums and sqrt are monotone, so the bounds hold for
// the rounded canonical values too).  ti = (wlo, whi, flags, b) with flags
// bit0 = dead (whole window before the oldest slice), bit1 = near (some pair
// may be screened), bit2 = some pair lies before slot -2 (its floor position
// must be clamped to the window's slot -2 entry: zero, or the held slice 0
// with zero derivative), bits 8..15 = valid cells;
// tf = brick corner relative to
// the tile reference in FP32, in units of c dt, and (bit pattern of tf.w) the
// brick row by + nby * bz; cc = canonical x0, x1, y0, y1, z0, z1.
template <class PP>
__device__ __forceinline__ void brick_info(const PP& p, const TileGeom& g, int b, int b_end,
                                           int4& ti, float4& tf, double cc[6]) {
  ti = make_int4(0, -1, 1, b);
  tf = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int q = 0; q < 6; ++q) cc[q] = 0.0;
  if (b >= b_end) return;
  const int bz = b / (p.nbx * p.nby);
  const int by = (b / p.nbx) % p.nby;
  const int bx = b % p.nbx;
  const int i0 = 2 * bx, j0 = 2 * by, k0 = 2 * bz;
  const int i1 = min(i0 + 1, p.src.n[0] - 1);
  const int j1 = min(j0 + 1, p.src.n[1] - 1);
  const int k1 = min(k0 + 1, p.src.n[2] - 1);
  cc[0] = canon(p.src.o[0], i0, p.src.h[0]);
  cc[1] = canon(p.src.o[0], i1, p.src.h[0]);
  cc[2] = canon(p.src.o[1], j0, p.src.h[1]);
  cc[3] = canon(p.src.o[1], j1, p.src.h[1]);
  cc[4] = canon(p.src.o[2], k0, p.src.h[2]);
  cc[5] = canon(p.src.o[2], k1, p.src.h[2]);
  const double blo[3] = {cc[0], cc[2], cc[4]};
  const double bhi[3] = {cc[1], cc[3], cc[5]};
  const double tlo[3] = {g.refx, g.refy, g.refz};
  const double thi[3] = {g.thix, g.thiy, g.thiz};
  double g2 = 0.0, f2 = 0.0;
  bool near = true;
  for (int a = 0; a < 3; ++a) {
    const double gap = __builtin_fmax(0.0, __builtin_fmax(blo[a] - thi[a], tlo[a] - bhi[a]));
    const double far = __builtin_fmax(bhi[a] - tlo[a], thi[a] - blo[a]);
    g2 += gap * gap;
    f2 += far * far;
    near = near && (gap <= p.screen[a] + p.near_slack);
  }
  // correctly rounded square roots: the bounds then hold for the rounded
  // canonical values by monotonicity (the hardware v_sqrt_f64 alone is far
  // less accurate than the margin)
  const double ulo = p.a_f - __builtin_sqrt(f2) * p.inv_cdt - p.margin;
  const double uhi = p.a_f - __builtin_sqrt(g2) * p.inv_cdt + p.margin;
  const int jlo = p.a_i + (int)__builtin_fmax(__builtin_floor(ulo), -1e9);
  int jhi = p.a_i + (int)__builtin_fmax(__builtin_floor(uhi), -1e9);
  jhi = min(jhi, p.nt - 1);
  // held past: a window wholly before slice -1 still reads the held values
  // through its clamp entry, so no brick is dead
  const bool hold = (p.stencil & kStencilHold) != 0;
  if (hold) jhi = max(jhi, -2);
  const bool dead = !hold && jhi < -1;
  // cells with cx = 1 (cy = 1, cz = 1) exist when the brick has two layers in x (y, z)
  const int vmask = (i1 > i0 ? 0xff : 0x55) & (j1 > j0 ? 0xff : 0x33) & (k1 > k0 ? 0xff : 0x0f);
  ti = make_int4(max(jlo, -2), jhi, (dead ? 1 : 0) | (near ? 2 : 0) | (jlo < -2 ? 4 : 0) | (vmask << 8), b);
  tf = make_float4((float)((cc[0] - g.refx) * p.inv_cdt), (float)((cc[2] - g.refy) * p.inv_cdt),
                   (float)((cc[4] - g.refz) * p.inv_cdt), __int_as_float(by + p.nby * bz));
}

template <typename T, int G, bool FP, bool MULTI>
__global__ __launch_bounds__(kThreads) void pair_kernel(PairParams p) {
  constexpr int NPL = Traits<T>::kPlanes;
  constexpr int CELLS = G * kBrickCells;
  constexpr int PU = CELLS * kWmax;  // 16-byte units per plane
  __shared__ float4 lds[NPL * PU];
  __shared__ int4 tab_i[G];
  __shared__ float4 tab_f[G];
  __shared__ double tab_c[G][6];

  const int bid = xcd_remap((int)blockIdx.x, p.n_wg, p.n_tiles, p.n_splits);
  const int split = bid / p.n_tiles;
  const int tile = bid - split * p.n_tiles;
  const TileGeom tg = tile_geom(p, tile);
  const int ix0 = tg.ix0, iy0 = tg.iy0, iz0 = tg.iz0;
  const int ix1 = tg.ix1, iy1 = tg.iy1, iz1 = tg.iz1;
  const int t = (int)threadIdx.x;
  const int w = t >> 6, l = t & 63;
  const int ix = ix0 + (w & 1) * 4 + (l & 3);
  const int iy = iy0 + ((w >> 1) & 1) * 4 + ((l >> 2) & 3);
  const int iz = iz0 + (w >> 2) * 4 + (l >> 4);
  const bool valid = ix <= ix1 && iy <= iy1 && iz <= iz1;
  const int cix = min(ix, ix1), ciy = min(iy, iy1), ciz = min(iz, iz1);

  const double refx = tg.refx, refy = tg.refy, refz = tg.refz;
  const double rox = canon(p.obs.o[0], cix, p.obs.h[0]);
  const double roy = canon(p.obs.o[1], ciy, p.obs.h[1]);
  const double roz = canon(p.obs.o[2], ciz, p.obs.h[2]);

  const T* ring = (const T*)p.ring;
  const int b_begin = split * p.bricks_per_split;
  const int b_end = min(b_begin + p.bricks_per_split, p.n_bricks);

  // accumulators
  float sE[3] = {0.f, 0.f, 0.f}, cE[3] = {0.f, 0.f, 0.f};
  float sB[3] = {0.f, 0.f, 0.f}, cB[3] = {0.f, 0.f, 0.f};
  double dE[3] = {0.0, 0.0, 0.0}, dB[3] = {0.0, 0.0, 0.0};
  unsigned long long n_live = 0, sum_k = 0, sum_kw = 0, n_scr = 0;

  // FP32 arithmetic works in units of c dt (lengths scaled by 1/(c dt), time
  // derivatives by dt); the prefactor of the FP32 plan scales the sums back
  const double ls = p.inv_cdt;
  const float xo = (float)((rox - refx) * ls), yo = (float)((roy - refy) * ls), zo = (float)((roz - refz) * ls);
  const float hsx = (float)(p.src.h[0] * ls), hsy = (float)(p.src.h[1] * ls), hsz = (float)(p.src.h[2] * ls);
  const float af32 = (float)p.a_f, halfg = 0.5f - p.guard;
  const T inv_dt = sizeof(T) == 4 ? (T)(p.inv_dt / p.inv_cdt) : (T)p.inv_dt;

  for (int rb = b_begin; rb < b_end; rb += G) {
    __syncthreads();  // the previous round's readers are done with LDS and the table
    if (t < G) {
      int4 ti;
      float4 tf;
      double cc[6];
      brick_info(p, tg, rb + t, b_end, ti, tf, cc);
      tab_i[t] = ti;
      tab_f[t] = tf;
      for (int q = 0; q < 6; ++q) tab_c[t][q] = cc[q];
    }
    __syncthreads();

    int n_chunks = 1;
    if (MULTI) {
      int wmax_round = 0;
      for (int j = 0; j < G; ++j) {
        const int4 ti = tab_i[j];
        if (!(ti.z & 1)) wmax_round = max(wmax_round, ti.y - ti.x + 1);
      }
      n_chunks = (wmax_round + kWmax - 1) / kWmax;
      if (FP) n_chunks = max(n_chunks, 1);  // screened pairs of dead bricks are still counted
    }

    for (int ch = 0; ch < n_chunks; ++ch) {
      const int cs = ch * kWmax;
      if (ch > 0) __syncthreads();
      // ---- stage the slice windows of this round's bricks into LDS ----
      for (int it = t; it < G * kWmax * kBrickCells; it += kThreads) {
        const int c = it & 7;
        const int kk = (it >> 3) % kWmax;
        const int j = (it >> 3) / kWmax;
        const int4 ti = tab_i[j];
        if (ti.z & 1) continue;
        const int k = ti.x + cs + kk;
        if (k > ti.y) continue;
        const int e = (j * kBrickCells + c) * kWmax + kk;
        typename RawOf<T>::type hm, h0, h1;
        load_raw(ring, p, k - 1, ti.w, c, hm);
        load_raw(ring, p, k, ti.w, c, h0);
        load_raw(ring, p, k + 1, ti.w, c, h1);
        // a history that starts at slice 0 keeps no value before it (the
        // held reads make every other plane zero there)
        const bool value = k >= 0 || !(p.stencil & kStencilCut);
        if (p.stencil & kStencilCubic) {
          typename RawOf<T>::type h2;
          load_raw(ring, p, k - 2, ti.w, c, h2);
          put_cubic(lds, PU, e, h2, hm, h0, h1, value);
        } else if (p.stencil & kStencilSlope)
          put_entry<true>(lds, PU, e, hm, h0, h1, inv_dt, value);
        else
          put_entry<false>(lds, PU, e, hm, h0, h1, inv_dt, value);
      }
      __syncthreads();

      // ---- pair loop over this round's source cells ----
      float bE[3] = {0.f, 0.f, 0.f}, bB[3] = {0.f, 0.f, 0.f};
      for (int j = 0; j < G; ++j) {
        const int4 ti = tab_i[j];
        const bool dead = (ti.z & 1) != 0;
        // the fingerprint pass counts the screened pairs of dead near bricks too
        if (dead && !(FP && (ti.z & 2))) continue;
        const float4 tf = tab_f[j];
        const bool near = (ti.z & 2) != 0;
        const int vmask = ti.z >> 8;
        const int lo_c = ti.x + cs;
        const int hi_c = min(ti.y, lo_c + kWmax - 1);
        const int base = j * kBrickCells * kWmax - lo_c;
        const float d0x = xo - tf.x, d0y = yo - tf.y, d0z = zo - tf.z;
        double bc[6];
        if constexpr (sizeof(T) == 8) {
          for (int q = 0; q < 6; ++q) bc[q] = tab_c[j][q];
        }
        int s_base = 0;
        if (FP) {
          const int b = ti.w;
          const int bz = b / (p.nbx * p.nby);
          const int by = (b / p.nbx) % p.nby;
          const int bx = b % p.nbx;
          s_base = 2 * bx + p.src.n[0] * (2 * by + p.src.n[1] * 2 * bz);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if (!((vmask >> c) & 1)) continue;
          const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
          bool act = true;
          if (near) {
            const double ddx = rox - tab_c[j][cx];
            const double ddy = roy - tab_c[j][2 + cy];
            const double ddz = roz - tab_c[j][4 + cz];  // near bricks only
            if (canon_screened(ddx, ddy, ddz, p.screen)) {
              act = false;
              if (FP && cs == 0) n_scr += 1;
            }
          }
          if (!act || dead) continue;
          if constexpr (sizeof(T) == 4) {
            const float dx = cx ? d0x - hsx : d0x;
            const float dy = cy ? d0y - hsy : d0y;
            const float dz = cz ? d0z - hsz : d0z;
            float m, f, ri;
            index_f32(dx, dy, dz, af32, halfg,
                      [&]() {
                        return canon_u(rox - tab_c[j][cx], roy - tab_c[j][2 + cy],
                                       roz - tab_c[j][4 + cz], p.a_f, p.inv_cdt);
                      },
                      m, f, ri);
            const int k = p.a_i + (int)m;
            const int kc = min(max(k, ti.x), MULTI ? ti.y : hi_c);
            if (MULTI && (kc < lo_c || kc > hi_c)) continue;
            if (FP) {
              if (k >= -1) {
                const int s = s_base + cx + p.src.n[0] * (cy + p.src.n[1] * cz);
                n_live += 1;
                sum_k += (unsigned long long)(long long)k;
                sum_kw += (unsigned long long)(long long)k * (unsigned long long)(s + 1);
              }
              continue;
            }
            const int e = base + c * kWmax + kc;
            const float ri2 = ri * ri;
            const float ri3 = ri2 * ri;
            float v[4], w[4];
            if (p.stencil & kStencilCubic)
              entry_at<true>(lds, PU, e, f, inv_dt, v, w);
            else
              entry_at<false>(lds, PU, e, f, inv_dt, v, w);
            const float rho = v[0], jx = v[1], jy = v[2], jz = v[3];
            const float rhod = w[0], jdx = w[1], jdy = w[2], jdz = w[3];
            const float a = __builtin_fmaf(rho, ri3, rhod * ri2);
            bE[0] = __builtin_fmaf(dx, a, bE[0]);
            bE[1] = __builtin_fmaf(dy, a, bE[1]);
            bE[2] = __builtin_fmaf(dz, a, bE[2]);
            bE[0] = __builtin_fmaf(-jdx, ri, bE[0]);
            bE[1] = __builtin_fmaf(-jdy, ri, bE[1]);
            bE[2] = __builtin_fmaf(-jdz, ri, bE[2]);
            const float Kx = __builtin_fmaf(jx, ri3, jdx * ri2);
            const float Ky = __builtin_fmaf(jy, ri3, jdy * ri2);
            const float Kz = __builtin_fmaf(jz, ri3, jdz * ri2);
            bB[0] = __builtin_fmaf(Ky, dz, bB[0]);
            bB[0] = __builtin_fmaf(-Kz, dy, bB[0]);
            bB[1] = __builtin_fmaf(Kz, dx, bB[1]);
            bB[1] = __builtin_fmaf(-Kx, dz, bB[1]);
            bB[2] = __builtin_fmaf(Kx, dy, bB[2]);
            bB[2] = __builtin_fmaf(-Ky, dx, bB[2]);
          } else {
            const double dx = rox - bc[cx];
            const double dy = roy - bc[2 + cy];
            const double dz = roz - bc[4 + cz];
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            const double R = __builtin_sqrt(r2);
            const double u = p.a_f - R * p.inv_cdt;
            const double m = __builtin_fmax(__builtin_floor(u), -1e9);
            const double f = u - m;
            const int k = p.a_i + (int)m;
            const int kc = min(max(k, ti.x), MULTI ? ti.y : hi_c);
            if (MULTI && (kc < lo_c || kc > hi_c)) continue;
            if (FP) {
              if (k >= -1) {
                const int s = s_base + cx + p.src.n[0] * (cy + p.src.n[1] * cz);
                n_live += 1;
                sum_k += (unsigned long long)(long long)k;
                sum_kw += (unsigned long long)(long long)k * (unsigned long long)(s + 1);
              }
              continue;
            }
            // 1/R: hardware reciprocal refined by two Newton steps
            double ri = __builtin_amdgcn_rcp(R);
            double er = __builtin_fma(-R, ri, 1.0);
            ri = __builtin_fma(ri, er, ri);
            er = __builtin_fma(-R, ri, 1.0);
            ri = __builtin_fma(ri, er, ri);
            const double ri2 = ri * ri;
            const double ri3 = ri2 * ri;
            const int e = base + c * kWmax + kc;
            double v[4], w[4];
            if (p.stencil & kStencilCubic)
              entry_at<true>(lds, PU, e, f, (double)inv_dt, v, w);
            else
              entry_at<false>(lds, PU, e, f, (double)inv_dt, v, w);
            const double rho = v[0], jx = v[1], jy = v[2], jz = v[3];
            const double rhod = w[0], jdx = w[1], jdy = w[2], jdz = w[3];
            const double a = __builtin_fma(rho, ri3, rhod * ri2);
            dE[0] = __builtin_fma(dx, a, dE[0]);
            dE[1] = __builtin_fma(dy, a, dE[1]);
            dE[2] = __builtin_fma(dz, a, dE[2]);
            dE[0] = __builtin_fma(-jdx, ri, dE[0]);
            dE[1] = __builtin_fma(-jdy, ri, dE[1]);
            dE[2] = __builtin_fma(-jdz, ri, dE[2]);
            const double Kx = __builtin_fma(jx, ri3, jdx * ri2);
            const double Ky = __builtin_fma(jy, ri3, jdy * ri2);
            const double Kz = __builtin_fma(jz, ri3, jdz * ri2);
            dB[0] = __builtin_fma(Ky, dz, dB[0]);
            dB[0] = __builtin_fma(-Kz, dy, dB[0]);
            dB[1] = __builtin_fma(Kz, dx, dB[1]);
            dB[1] = __builtin_fma(-Kx, dz, dB[1]);
            dB[2] = __builtin_fma(Kx, dy, dB[2]);
            dB[2] = __builtin_fma(-Ky, dx, dB[2]);
          }
        }
      }
      if constexpr (sizeof(T) == 4) {
        if (!FP) {
          for (int a = 0; a < 3; ++a) {
            two_sum_acc(sE[a], cE[a], bE[a]);
            two_sum_acc(sB[a], cB[a], bB[a]);
          }
        }
      }
    }
  }

  if (!valid) return;
  const long long n_obs = (long long)p.obs.n[0] * p.obs.n[1] * p.obs.n[2];
  const long long o = (long long)ix + (long long)p.obs.n[0] * ((long long)iy + (long long)p.obs.n[1] * iz);
  if (FP) {
    atomicAdd(&p.fp[o * 4 + 0], n_live);
    atomicAdd(&p.fp[o * 4 + 1], sum_k);
    atomicAdd(&p.fp[o * 4 + 2], sum_kw);
    atomicAdd(&p.fp[o * 4 + 3], n_scr);
    return;
  }
  double tot[6];
  if constexpr (sizeof(T) == 4) {
    for (int a = 0; a < 3; ++a) {
      tot[a] = (double)sE[a] + (double)cE[a];
      tot[3 + a] = (double)sB[a] + (double)cB[a];
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      tot[a] = dE[a];
      tot[3 + a] = dB[a];
    }
  }
  if (p.direct) {
    for (int a = 0; a < 3; ++a) {
      const double e = tot[a] * p.pref, bb = tot[3 + a] * p.pref;
      if (p.out_f64) {
        ((double*)p.E)[a * n_obs + o] = e;
        ((double*)p.B)[a * n_obs + o] = bb;
      } else {
        ((float*)p.E)[a * n_obs + o] = (float)e;
        ((float*)p.B)[a * n_obs + o] = (float)bb;
      }
    }
  } else {
    for (int a = 0; a < 6; ++a) p.partial[((long long)split * 6 + a) * n_obs + o] = tot[a];
  }
}


// ---------------------------------------------------------------------------
// Fast pair kernel: every slice window of the launch fits one LDS staging
// chunk.  Per round of G bricks: the raw slices of the next round are loaded
// into registers while the current round is computed; LDS holds (h, S, D, T)
// planes of [cell][slot] entries with one pad entry per cell.  Full bricks
// outside the screening range take a two-phase path: slice decisions for all
// 8 cells first (one divergent FP64 fix-up if any falls in the guard band),
// then branch-free LDS reads and field arithmetic.

// Field contribution of one pair from its LDS entry (FP32).
template <bool CUB>
__device__ __forceinline__ void pair_fields(const float4* lds, int PU, int e, float f, float ri, float dx,
                                            float dy, float dz, float bE[3], float bB[3], float dsc) {
  float v[4], w[4];
  entry_at<CUB>(lds, PU, e, f, dsc, v, w);
  const float rho = v[0], jx = v[1], jy = v[2], jz = v[3];
  const float rhod = w[0], jdx = w[1], jdy = w[2], jdz = w[3];
  // E += d/R^2 (rho/R + rho_dot) - J_dot/R ;  B += (J/R + J_dot) x d/R^2
  const float ri2 = ri * ri;
  const float ux = dx * ri2, uy = dy * ri2, uz = dz * ri2;
  const float ap = __builtin_fmaf(rho, ri, rhod);
  bE[0] = __builtin_fmaf(ux, ap, bE[0]);
  bE[1] = __builtin_fmaf(uy, ap, bE[1]);
  bE[2] = __builtin_fmaf(uz, ap, bE[2]);
  bE[0] = __builtin_fmaf(-jdx, ri, bE[0]);
  bE[1] = __builtin_fmaf(-jdy, ri, bE[1]);
  bE[2] = __builtin_fmaf(-jdz, ri, bE[2]);
  const float Lx = __builtin_fmaf(jx, ri, jdx);
  const float Ly = __builtin_fmaf(jy, ri, jdy);
  const float Lz = __builtin_fmaf(jz, ri, jdz);
  bB[0] = __builtin_fmaf(Ly, uz, bB[0]);
  bB[0] = __builtin_fmaf(-Lz, uy, bB[0]);
  bB[1] = __builtin_fmaf(Lz, ux, bB[1]);
  bB[1] = __builtin_fmaf(-Lx, uz, bB[1]);
  bB[2] = __builtin_fmaf(Lx, uy, bB[2]);
  bB[2] = __builtin_fmaf(-Ly, ux, bB[2]);
}

// 1/R in FP64: hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double recip_f64(double R) {
  double ri = __builtin_amdgcn_rcp(R);
  double er = __builtin_fma(-R, ri, 1.0);
  ri = __builtin_fma(ri, er, ri);
  er = __builtin_fma(-R, ri, 1.0);
  return __builtin_fma(ri, er, ri);
}

// 1/sqrt(r2) in FP64: hardware estimate (about 2^-23 relative) and two
// Newton steps y += y (1/2 - (r2/2) y^2), each squaring the relative error.
__device__ __forceinline__ double rsqrt_f64(double r2) {
  double y = __builtin_amdgcn_rsq(r2);
  const double hr = 0.5 * r2;
  double e = __builtin_fma(-hr, y * y, 0.5);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-hr, y * y, 0.5);
  return __builtin_fma(y, e, y);
}

// Field contribution of one pair from the planes of its entry (FP64); ri = 1/R.
template <bool CUB>
__device__ __forceinline__ void pair_fields_from(const double P[4][4], double f, double ri, double dx, double dy,
                                                 double dz, double dE[3], double dB[3], double dsc) {
  double v[4], w[4];
  entry_from<CUB>(P, f, dsc, v, w);
  const double rho = v[0], jx = v[1], jy = v[2], jz = v[3];
  const double rhod = w[0], jdx = w[1], jdy = w[2], jdz = w[3];
  const double ri2 = ri * ri;
  const double ux = dx * ri2, uy = dy * ri2, uz = dz * ri2;
  const double ap = __builtin_fma(rho, ri, rhod);
  dE[0] = __builtin_fma(ux, ap, dE[0]);
  dE[1] = __builtin_fma(uy, ap, dE[1]);
  dE[2] = __builtin_fma(uz, ap, dE[2]);
  dE[0] = __builtin_fma(-jdx, ri, dE[0]);
  dE[1] = __builtin_fma(-jdy, ri, dE[1]);
  dE[2] = __builtin_fma(-jdz, ri, dE[2]);
  const double Lx = __builtin_fma(jx, ri, jdx);
  const double Ly = __builtin_fma(jy, ri, jdy);
  const double Lz = __builtin_fma(jz, ri, jdz);
  dB[0] = __builtin_fma(Ly, uz, dB[0]);
  dB[0] = __builtin_fma(-Lz, uy, dB[0]);
  dB[1] = __builtin_fma(Lz, ux, dB[1]);
  dB[1] = __builtin_fma(-Lx, uz, dB[1]);
  dB[2] = __builtin_fma(Lx, uy, dB[2]);
  dB[2] = __builtin_fma(-Ly, ux, dB[2]);
}

template <bool CUB>
__device__ __forceinline__ void pair_fields(const float4* lds, int PU, int e, double f, double ri, double dx,
                                            double dy, double dz, double dE[3], double dB[3], double dsc) {
  double P[4][4];
  planes_at(lds, PU, e, P);
  pair_fields_from<CUB>(P, f, ri, dx, dy, dz, dE, dB, dsc);
}

struct FpAcc {
  unsigned long long n_live = 0, sum_k = 0, sum_kw = 0, n_scr = 0;
  __device__ __forceinline__ void add(int k, int s) {
    if (k >= -1) {
      n_live += 1;
      sum_k += (unsigned long long)(long long)k;
      sum_kw += (unsigned long long)(long long)k * (unsigned long long)(s + 1);
    }
  }
};

// Table entries of live bricks waiting for their round (a power of two).
constexpr int kBrickRing = 64;

// A live brick's table entry: window and flags, and its FP32 corner and
// row (brick_info), side by side so that one address serves both reads.
struct BrickEntry {
  int4 i;
  float4 f;
};

// Launch shape: WZ = 1 (8x8x4 tiles, 256 threads) or 2 (8x8x8, 512 threads);
// W = slots staged per cell (32, 64 or 128) -- the longer the window, the
// fewer bricks fit a round in the same LDS.
template <typename T, int WZ, int W>
struct FastShape {
  static constexpr int G = (sizeof(T) == 4 ? 2 : 1) * WZ * 32 / W;  // bricks per round
  static constexpr int KT = 256 * WZ;                                // threads
  static constexpr int NPL = Traits<T>::kPlanes;
  static constexpr int CS = W + 1;                           // cell stride in entries (one pad entry)
  static constexpr int PU = G * kBrickCells * CS;            // 16-byte units per plane
  static constexpr int THR = sizeof(T) == 4 ? kThrMax : kThrMax64;
  static_assert(G >= 1, "window too long for this shape");
};

// One workgroup's share of a launch: tile x source split number `bid` of
// the problem described by p.
// IDX (FP32 only): 0 = FP32 index with guard band and FP64 re-decision,
// 1 = threshold-table decision for every pair of a full brick.  PP is
// PairParams as a kernel argument, or in the constant address space for
// the persistent kernel (uniform, read-only: scalar loads).  STG: staging
// mode, bit 0 = cubic planes, bit 1 = a history that starts at slice 0 (its
// own instantiations, so the other kernels' code is unchanged by it).
template <typename T, int WZ, bool FP, int IDX, int W, int STG, class PP>
__device__ __forceinline__ void pair_body(const PP& p, int bid,
                                          float4 (&lds)[FastShape<T, WZ, W>::NPL * FastShape<T, WZ, W>::PU],
                                          BrickEntry (&tab)[kBrickRing],
                                          double (&tab_c)[kBrickRing][6],
                                          double (&thr)[FastShape<T, WZ, W>::THR], int (&qs)[2]) {
  using Raw = typename RawOf<T>::type;
  constexpr bool CUB = (STG & 1) != 0;
  constexpr bool PCUT = (STG & 2) != 0;
  constexpr int G = FastShape<T, WZ, W>::G;
  constexpr int kThreads = FastShape<T, WZ, W>::KT;
  constexpr int PU = FastShape<T, WZ, W>::PU;
  constexpr int kCellStride = FastShape<T, WZ, W>::CS;
  constexpr int EPT = G * kBrickCells * W / kThreads;  // staged entries per thread
  constexpr int NRAW = EPT + (CUB ? 3 : 2);  // raw slices k0-1 (k0-2 for the cubic) .. k0+EPT
  constexpr int NQ = W / EPT;
  static_assert(EPT >= 1 && EPT * kThreads == G * kBrickCells * W, "staging map");

  const int split = bid / p.n_tiles;
  const int tile = bid - split * p.n_tiles;
  const TileGeom tg = tile_geom(p, tile);
  const int t = (int)threadIdx.x;
  if (p.use_thr)
    for (int i = t; i < p.thr_n; i += kThreads) thr[i] = p.thr[i];
  const int w = t >> 6, l = t & 63;
  const int ix = tg.ix0 + (w & 1) * 4 + (l & 3);
  const int iy = tg.iy0 + ((w >> 1) & 1) * 4 + ((l >> 2) & 3);
  const int iz = tg.iz0 + (w >> 2) * 4 + (l >> 4);
  const bool valid = ix <= tg.ix1 && iy <= tg.iy1 && iz <= tg.iz1;
  const bool wave_live = __any(valid);
  const int cix = min(ix, tg.ix1), ciy = min(iy, tg.iy1), ciz = min(iz, tg.iz1);
  const double rox = canon(p.obs.o[0], cix, p.obs.h[0]);
  const double roy = canon(p.obs.o[1], ciy, p.obs.h[1]);
  const double roz = canon(p.obs.o[2], ciz, p.obs.h[2]);
  // FP32 arithmetic works in units of c dt (lengths scaled by 1/(c dt), time
  // derivatives by dt); the prefactor of the FP32 plan scales the sums back
  const double ls = p.inv_cdt;
  const float xo = (float)((rox - tg.refx) * ls), yo = (float)((roy - tg.refy) * ls),
              zo = (float)((roz - tg.refz) * ls);
  const float hsx = (float)(p.src.h[0] * ls), hsy = (float)(p.src.h[1] * ls), hsz = (float)(p.src.h[2] * ls);
  const float af32 = (float)p.a_f, halfg = 0.5f - p.guard;
  const T inv_dt = sizeof(T) == 4 ? (T)(p.inv_dt / p.inv_cdt) : (T)p.inv_dt;
  const T* ring = (const T*)p.ring;
  // threshold of floor position N at thr_at[N]; N stays in the table's range
  const double* thr_at = &thr[0] - p.thr_lo;
  const int b_begin = split * p.bricks_per_split;
  const int b_end = min(b_begin + p.bricks_per_split, p.n_bricks);

  // staging assignment: cell fastest (coalesced 16-byte loads along a brick)
  const int sc = t & 7;
  const int sq = (t >> 3) % NQ;
  const int sj = (t >> 3) / NQ;

  float sE[3] = {0.f, 0.f, 0.f}, cE[3] = {0.f, 0.f, 0.f};
  float sB[3] = {0.f, 0.f, 0.f}, cB[3] = {0.f, 0.f, 0.f};
  double dE[3] = {0.0, 0.0, 0.0}, dB[3] = {0.0, 0.0, 0.0};
  FpAcc fpa;
  Raw raw[NRAW];

  // Live bricks wait in a ring of kBrickRing table entries (logical
  // positions, taken modulo the ring size): a round uses the next G of
  // them.  Wavefront 0 refills the ring when fewer than G wait for the
  // next round: it tests the 64 bricks from `cursor` on, one per lane, and
  // appends the live ones (dead bricks -- every pair before the oldest
  // slice -- take no round slot), as many as there is room for behind
  // `keep` (the oldest entry still in use).  qs receives the new tail and
  // the cursor after the last brick taken.
  auto refill = [&](int keep, int tail, int cursor) {
    if (t < 64) {
      int4 ti;
      float4 tf;
      double cc[6];
      brick_info(p, tg, cursor + t, b_end, ti, tf, cc);  // past b_end: a dead entry
      // the fingerprint pass also takes dead bricks that may hold screened
      // pairs: it counts every screened pair
      const bool live = !(ti.z & 1) || (FP && (ti.z & 2));
      const unsigned long long m = __ballot(live);
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      const int got = (int)__popcll(m);
      const int take = min(got, kBrickRing - (tail - keep));
      if (live && rank < take) {
        const int q = (tail + rank) & (kBrickRing - 1);
        tab[q].i = ti;
        tab[q].f = tf;
        for (int k = 0; k < 6; ++k) tab_c[q][k] = cc[k];
      }
      const unsigned long long last = __ballot(live && rank == take - 1);
      if (t == 0) {
        qs[0] = tail + take;
        qs[1] = min(take < got && last != 0ull ? cursor + (int)__builtin_ctzll(last) + 1 : cursor + 64, b_end);
      }
    }
  };
  // the round's brick slot j: entry pos + j when j < n, else a dead entry
  auto slot_entry = [&](int pos, int n, int j) {
    return j < n ? tab[(pos + j) & (kBrickRing - 1)].i : make_int4(0, -1, 1, 0);
  };
  // The 64 threads of a wavefront stage one brick slot (NQ is a multiple of
  // 8, so t >> 3 stays within one sj): the slot's table entry, its ring
  // slots and their range tests are uniform across the wavefront.
  static_assert(NQ % 8 == 0, "one brick slot per wavefront");
  const int sq0 = __builtin_amdgcn_readfirstlane(sq & ~7);  // first slot group of this wavefront
  const int sjw = __builtin_amdgcn_readfirstlane(sj);
  // per-lane part of a ring offset on the uniform path: slot group, cell
  const unsigned lane_off = (unsigned)((sq & 7) * EPT) * ((unsigned)p.slot_elems * (unsigned)sizeof(T)) +
                            (unsigned)sc * (4u * (unsigned)sizeof(T));
  auto load_round = [&](const int4& ti) {
    const int k0 = ti.x + sq * EPT;
    if (p.ring_bytes_rs != 0u) {
      // Buffer addressing over the ring: 32-bit offsets stepped slot by
      // slot, and slices outside 0..nt-1 read through an offset past the
      // end of the buffer, which the hardware returns as zero.
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc((void*)p.ring, (short)0, (int)p.ring_bytes_rs, kRawBufferFlags);
      const unsigned sb = (unsigned)p.slot_elems * (unsigned)sizeof(T);
      {
        // This wavefront's raw slices jw .. jw + SPAN - 1: when all lie in
        // 0..nt-1 and in consecutive ring slots, a scalar offset per slice.
        constexpr int SPAN = 7 * EPT + NRAW;
        const int jw = ti.x - (CUB ? 2 : 1) + sq0 * EPT;
        int slw = p.slot_base + jw;
        slw -= slw >= p.capacity ? p.capacity : 0;
        if (jw >= 0 && jw + SPAN <= p.nt && slw + SPAN <= p.capacity) {
          unsigned so = (unsigned)slw * sb + (unsigned)ti.w * (kBrickCells * 4u * (unsigned)sizeof(T));
#pragma unroll
          for (int r = 0; r < NRAW; ++r) {
            buffer_raw(rs, lane_off, so, raw[r]);
            so += sb;
          }
          return;
        }
      }
      const int j0 = k0 - (CUB ? 2 : 1);
      int sl = p.slot_base + j0;  // j0 >= -3 (-4 for the cubic)
      sl += sl < 0 ? p.capacity : 0;
      sl += sl < 0 ? p.capacity : 0;
      sl += sl < 0 ? p.capacity : 0;
      if constexpr (CUB) sl += sl < 0 ? p.capacity : 0;
      sl -= sl >= p.capacity ? p.capacity : 0;
      const unsigned cell_off = ((unsigned)ti.w * kBrickCells + (unsigned)sc) * (4u * (unsigned)sizeof(T));
      unsigned off = (unsigned)sl * sb + cell_off;
      if (p.stencil & (kStencilHold | kStencilCut)) {
        // slices before 0 read slice 0 (slot_base)
        const int o0 = (int)((unsigned)p.slot_base * sb + cell_off);
#pragma unroll
        for (int r = 0; r < NRAW; ++r) {
          const int j = j0 + r;
          const int o = j < 0 ? o0 : (j < p.nt ? (int)off : kOutOfRange);
          buffer_raw(rs, o, raw[r]);
          off += sb;
          off -= off >= p.ring_bytes_rs ? p.ring_bytes_rs : 0u;
        }
        return;
      }
#pragma unroll
      for (int r = 0; r < NRAW; ++r) {
        const int o = (unsigned)(j0 + r) < (unsigned)p.nt ? (int)off : kOutOfRange;
        buffer_raw(rs, o, raw[r]);
        off += sb;
        off -= off >= p.ring_bytes_rs ? p.ring_bytes_rs : 0u;
      }
      return;
    }
#pragma unroll
    for (int r = 0; r < NRAW; ++r) load_raw(ring, p, k0 - (CUB ? 2 : 1) + r, ti.w, sc, raw[r]);
  };
  auto write_round = [&](const int4& ti) {
    const int base = (sj * kBrickCells + sc) * kCellStride + sq * EPT;
    // A history that starts at slice 0: an entry of an earlier slice was
    // staged from the held slice 0 at every node, so all its planes but the
    // value are zero already; it keeps no value either.
    const int kv = PCUT ? -(ti.x + sq * EPT) : INT_MIN;  // entries e < kv lie before
    if constexpr (CUB) {
#pragma unroll
      for (int e = 0; e < EPT; ++e)
        put_cubic(lds, PU, base + e, raw[e], raw[e + 1], raw[e + 2], raw[e + 3], e >= kv);
    } else if (p.stencil & kStencilSlope) {
#pragma unroll
      for (int e = 0; e < EPT; ++e)
        put_entry<true>(lds, PU, base + e, raw[e], raw[e + 1], raw[e + 2], inv_dt, e >= kv);
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e)
        put_entry<false>(lds, PU, base + e, raw[e], raw[e + 1], raw[e + 2], inv_dt, e >= kv);
    }
  };

  int cursor = b_begin, tail = 0, pos = 0, cnt = 0;
  if (cursor < b_end) {
    refill(0, 0, cursor);
    __syncthreads();
    tail = __builtin_amdgcn_readfirstlane(qs[0]);  // uniform: keeps ring positions scalar
    cursor = __builtin_amdgcn_readfirstlane(qs[1]);
    cnt = min(G, tail);
  }
  // Source-cell index of a brick's first cell (fingerprints only).
  auto brick_s_base = [&](int b) {
    const int bz = b / (p.nbx * p.nby);
    const int by = (b / p.nbx) % p.nby;
    const int bx = b % p.nbx;
    return 2 * bx + p.src.n[0] * (2 * by + p.src.n[1] * 2 * bz);
  };
  auto cell_s = [&](int s_base, int c) {
    return s_base + (c & 1) + p.src.n[0] * (((c >> 1) & 1) + p.src.n[1] * (c >> 2));
  };

  // rounds continue while bricks remain: the round uses ring entries
  // pos .. pos + cnt - 1; bricks from `cursor` on are not yet tested
  // FP32 block sums of two rounds (up to 64 pairs per lane), then an
  // error-free two-sum into the running totals
  float bE[3] = {0.f, 0.f, 0.f}, bB[3] = {0.f, 0.f, 0.f};
  int n_blk = 0;
  // y and z parts of the full-brick geometry, kept while consecutive bricks
  // lie in one brick row (the same y and z cells): FP32 separations and
  // sums of squares, canonical FP64 squares
  int row_key = -1;
  float sy0 = 0.f, sy1 = 0.f, sz0 = 0.f, sz1 = 0.f, yzs[4] = {0.f, 0.f, 0.f, 0.f};
  double ey2s[2] = {0.0, 0.0}, ez2s[2] = {0.0, 0.0};
  // FP64 full bricks: the y and z separations and squares of the last brick row
  double rey[2] = {0.0, 0.0}, rez[2] = {0.0, 0.0}, ry2[2] = {0.0, 0.0}, rz2[2] = {0.0, 0.0};
  for (bool more = b_begin < b_end; more;) {
    // each round loads its raw slices at its start: holding the next round's
    // in registers while this one computes costs the pair loop more (spills)
    // than the loads' latency
    {
      const int4 tv = slot_entry(pos, cnt, sjw);
      const int4 ti = make_int4(__builtin_amdgcn_readfirstlane(tv.x), 0, __builtin_amdgcn_readfirstlane(tv.z),
                                __builtin_amdgcn_readfirstlane(tv.w));
      // nothing to stage for an empty or dead brick slot
      if (!(ti.z & 1)) {
        load_round(ti);
        write_round(ti);
      }
    }
    const int npos = pos + cnt;
    const bool probe = tail - npos < G && cursor < b_end;
    if (probe) refill(pos, tail, cursor);
    __syncthreads();
    if (probe) {
      tail = __builtin_amdgcn_readfirstlane(qs[0]);  // uniform: keeps ring positions scalar
      cursor = __builtin_amdgcn_readfirstlane(qs[1]);
    }
    const int ncnt = min(G, tail - npos);
    const bool next = ncnt > 0 || cursor < b_end;

    // a wavefront whose 4x4x4 block lies wholly outside the observation
    // grid (tile padding) stages but computes nothing
    if (wave_live) {
    if constexpr (sizeof(T) == 4) {
      // Full far bricks first (all 8 cells, no screening possible), then the
      // rest (missing cells or possibly screened pairs) in a second pass.
      unsigned slow = 0;
#pragma unroll 1
      for (int j = 0; j < cnt; ++j) {
        const int q = (pos + j) & (kBrickRing - 1);
        const BrickEntry be = tab[q];
        const int tz = __builtin_amdgcn_readfirstlane(be.i.z);
        if (tz & 1) {
          if (FP && (tz & 2)) slow |= 1u << j;  // fingerprint: count its screened pairs
          continue;
        }
        if ((tz & 0xff02) != 0xff00) {
          slow |= 1u << j;
          continue;
        }
        const int4 ti = be.i;
        // window slot of floor position m: m + off
        const int off = __builtin_amdgcn_readfirstlane(p.a_i - ti.x);
        const int cellbase = j * kBrickCells * kCellStride + off;
        const int mlo = -off;
        const double* bc = tab_c[q];
        const float4 tf = be.f;
        const int row = __builtin_amdgcn_readfirstlane(__float_as_int(tf.w));
        if (row != row_key) {
          row_key = row;
          sy0 = yo - tf.y;
          sz0 = zo - tf.z;
          sy1 = sy0 - hsy;
          sz1 = sz0 - hsz;
          const float y2[2] = {sy0 * sy0, sy1 * sy1};
          const float z2[2] = {sz0 * sz0, sz1 * sz1};
          yzs[0] = y2[0] + z2[0];
          yzs[1] = y2[1] + z2[0];
          yzs[2] = y2[0] + z2[1];
          yzs[3] = y2[1] + z2[1];
          if constexpr (IDX == 1) {
            const double ey[2] = {roy - bc[2], roy - bc[3]};
            const double ez[2] = {roz - bc[4], roz - bc[5]};
            ey2s[0] = ey[0] * ey[0];
            ey2s[1] = ey[1] * ey[1];
            ez2s[0] = ez[0] * ez[0];
            ez2s[1] = ez[1] * ez[1];
          }
        }
        const float d0x = xo - tf.x, d1x = d0x - hsx;
        const float d0y = sy0, d1y = sy1, d0z = sz0, d1z = sz1;
        const float x2[2] = {d0x * d0x, d1x * d1x};
        float ri[8], fr[8], uu[8];
        int m[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const float r2 = x2[c & 1] + yzs[c >> 1];
          ri[c] = __builtin_amdgcn_rsqf(r2);
          uu[c] = __builtin_fmaf(-r2, ri[c], af32);
        }
        if constexpr (IDX == 1) {
          // Every pair: N = nearest integer to u32, then floor(u64) = N when
          // the canonical r2 <= T(N), else N - 1 (|u32 - u64| < 1/2).
          int nn[8];
          double tn[8];
#pragma unroll
          for (int c = 0; c < 8; ++c) nn[c] = cvt_nearest(uu[c]);
#pragma unroll
          for (int c = 0; c < 8; ++c) tn[c] = thr_at[nn[c]];
          const double ex[2] = {rox - bc[0], rox - bc[1]};
          const double ex2[2] = {ex[0] * ex[0], ex[1] * ex[1]};
          // canonical r2 = (dx*dx + dy*dy) + dz*dz
          const double exy[4] = {ex2[0] + ey2s[0], ex2[1] + ey2s[0], ex2[0] + ey2s[1], ex2[1] + ey2s[1]};
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int mn = exy[c & 3] + ez2s[c >> 2] <= tn[c] ? nn[c] : nn[c] - 1;
            m[c] = mn;
            fr[c] = uu[c] - (float)mn;
          }
        } else {
          bool risky = false;
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const float fl = __builtin_floorf(uu[c]);
            fr[c] = uu[c] - fl;
            m[c] = (int)fl;
            risky = risky || !(__builtin_fabsf(fr[c] - 0.5f) <= halfg);
          }
          if (risky) {
            if (p.use_thr) {
              // canonical r2 = (dx*dx + dy*dy) + dz*dz, parts shared by the 8 cells
              const double ex[2] = {rox - bc[0], rox - bc[1]};
              const double ey[2] = {roy - bc[2], roy - bc[3]};
              const double ez[2] = {roz - bc[4], roz - bc[5]};
              const double ez2[2] = {ez[0] * ez[0], ez[1] * ez[1]};
              const double exy[4] = {ex[0] * ex[0] + ey[0] * ey[0], ex[1] * ex[1] + ey[0] * ey[0],
                                     ex[0] * ex[0] + ey[1] * ey[1], ex[1] * ex[1] + ey[1] * ey[1]};
#pragma unroll
              for (int c = 0; c < 8; ++c) {
                if (!(__builtin_fabsf(fr[c] - 0.5f) <= halfg)) {
                  const double r2 = exy[c & 3] + ez2[c >> 2];
                  const int N = m[c] + (fr[c] > 0.5f ? 1 : 0);
                  const int mn = r2 <= thr[min(max(N - p.thr_lo, 0), p.thr_n - 1)] ? N : N - 1;
                  fr[c] += (float)(m[c] - mn);
                  m[c] = mn;
                }
              }
            } else {
#pragma unroll
              for (int c = 0; c < 8; ++c) {
                if (!(__builtin_fabsf(fr[c] - 0.5f) <= halfg)) {
                  const double u64 = canon_u(rox - bc[c & 1], roy - bc[2 + ((c >> 1) & 1)],
                                             roz - bc[4 + (c >> 2)], p.a_f, p.inv_cdt);
                  const double m64 = __builtin_floor(u64);
                  m[c] = (int)__builtin_fmax(m64, -1e9);
                  fr[c] = (float)(u64 - m64);
                }
              }
            }
          }
        }
        if (FP) {
          const int s_base = brick_s_base(ti.w);
#pragma unroll
          for (int c = 0; c < 8; ++c) fpa.add(p.a_i + m[c], cell_s(s_base, c));
          continue;
        }
        // m <= mhi holds by the window bounds; below mlo lies the zero
        // entry of pairs wholly before the oldest slice, which only bricks
        // flagged by bit 2 can have
        if (tz & 4) {
          // a brick straddling the switch-on front: skip it for this wavefront
          // when every pair lies before slice -1 (all contributions are zero,
          // unless the past is held)
          int mmax = m[0];
#pragma unroll
          for (int c = 1; c < 8; ++c) mmax = max(mmax, m[c]);
          if (!(p.stencil & kStencilHold) && !__any(mmax >= -1 - p.a_i)) continue;
#pragma unroll
          for (int c = 0; c < 8; ++c)
            pair_fields<CUB>(lds, PU, cellbase + c * kCellStride + max(m[c], mlo), fr[c], ri[c],
                             (c & 1) ? d1x : d0x, ((c >> 1) & 1) ? d1y : d0y, (c >> 2) ? d1z : d0z, bE, bB, inv_dt);
        } else {
#pragma unroll
          for (int c = 0; c < 8; ++c)
            pair_fields<CUB>(lds, PU, cellbase + c * kCellStride + m[c], fr[c], ri[c], (c & 1) ? d1x : d0x,
                             ((c >> 1) & 1) ? d1y : d0y, (c >> 2) ? d1z : d0z, bE, bB, inv_dt);
        }
      }
#pragma unroll 1
      for (int j = 0; slow != 0u; ++j, slow >>= 1) {
        if (!(slow & 1u)) continue;
        const int q = (pos + j) & (kBrickRing - 1);
        const int4 ti = tab[q].i;
        const int lo = ti.x;
        const int hiw = min(ti.y - lo, W - 1);
        const int off = p.a_i - lo;
        const int cellbase = __builtin_amdgcn_readfirstlane(j * kBrickCells * kCellStride + off);
        const int mlo = -off, mhi = hiw - off;
        const double* bc = tab_c[q];
        const float4 tf = tab[q].f;
        const float d0x = xo - tf.x, d0y = yo - tf.y, d0z = zo - tf.z;
        const float d1x = d0x - hsx, d1y = d0y - hsy, d1z = d0z - hsz;
        const int s_base = FP ? brick_s_base(ti.w) : 0;
        const int vmask = ti.z >> 8;
        const bool near = (ti.z & 2) != 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if (!((vmask >> c) & 1)) continue;
          const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
          if (near && canon_screened(rox - bc[cx], roy - bc[2 + cy], roz - bc[4 + cz], p.screen)) {
            if (FP) fpa.n_scr += 1;
            continue;
          }
          const float dx = cx ? d1x : d0x, dy = cy ? d1y : d0y, dz = cz ? d1z : d0z;
          float mf, f, ri;
          index_f32(dx, dy, dz, af32, halfg,
                    [&]() { return canon_u(rox - bc[cx], roy - bc[2 + cy], roz - bc[4 + cz], p.a_f, p.inv_cdt); },
                    mf, f, ri);
          const int mm = (int)mf;
          if (FP) {
            fpa.add(p.a_i + mm, cell_s(s_base, c));
            continue;
          }
          const int e = cellbase + c * kCellStride + min(max(mm, mlo), mhi);
          pair_fields<CUB>(lds, PU, e, f, ri, dx, dy, dz, bE, bB, inv_dt);
        }
      }
      if (!FP && (++n_blk & 1) == 0) {
        for (int a = 0; a < 3; ++a) {
          two_sum_acc(sE[a], cE[a], bE[a]);
          two_sum_acc(sB[a], cB[a], bB[a]);
          bE[a] = 0.f;
          bB[a] = 0.f;
        }
      }
    } else {
#pragma unroll 1
      for (int j = 0; j < cnt; ++j) {
        const int q = (pos + j) & (kBrickRing - 1);
        const int tz = __builtin_amdgcn_readfirstlane(tab[q].i.z);
        if ((tz & 1) && !(FP && (tz & 2))) continue;  // fingerprint: dead near bricks still count screening
        if (p.use_thr && (tz & 0xff02) == 0xff00) {
          // A full far brick: every pair's canonical floor position is N or
          // N - 1 for N the integer nearest u (u from a refined 1/sqrt, within
          // 1e-15 of the canonical value), and it is N iff the canonical r2 is
          // at most the threshold T(N): no correctly rounded square root.
          const int4 ti = tab[q].i;
          // window slot of floor position m: m + off (uniform, so that the clamp
          // below takes a scalar operand)
          const int off = __builtin_amdgcn_readfirstlane(p.a_i - ti.x);
          const int cellbase = __builtin_amdgcn_readfirstlane(j * kBrickCells * kCellStride + off);
          // below mlo lies the zero entry of pairs wholly before the oldest
          // slice (only bricks flagged by bit 2 have such pairs); one scalar,
          // so that each pair's clamp is a single max
          const int mlo = __builtin_amdgcn_readfirstlane((tz & 4) ? -off : INT_MIN);
          const double* bc = tab_c[q];
          const int row = __builtin_amdgcn_readfirstlane(__float_as_int(tab[q].f.w));
          if (row != row_key) {
            row_key = row;
            rey[0] = roy - bc[2];
            rey[1] = roy - bc[3];
            rez[0] = roz - bc[4];
            rez[1] = roz - bc[5];
            ry2[0] = rey[0] * rey[0];
            ry2[1] = rey[1] * rey[1];
            rz2[0] = rez[0] * rez[0];
            rz2[1] = rez[1] * rez[1];
          }
          const double ex[2] = {rox - bc[0], rox - bc[1]};
          const double* ey = rey;
          const double* ez = rez;
          const double x2[2] = {ex[0] * ex[0], ex[1] * ex[1]};
          const double* y2 = ry2;
          const double* z2 = rz2;
          if (!FP && (tz & 4) && !(p.stencil & kStencilHold)) {
            // straddling the switch-on front: skip the brick for this
            // wavefront when even its nearest cell lies wholly before slice -1
            // (FP addition is monotone, so this is the smallest pair r2)
            const double r2min = (__builtin_fmin(x2[0], x2[1]) + __builtin_fmin(y2[0], y2[1])) +
                                 __builtin_fmin(z2[0], z2[1]);
            if (!__any(r2min <= thr_at[max(-1 - p.a_i, p.thr_lo)])) continue;
          }
          const double exy[4] = {x2[0] + y2[0], x2[1] + y2[0], x2[0] + y2[1], x2[1] + y2[1]};
          const int s_base = FP ? brick_s_base(ti.w) : 0;
          // one z layer (four cells) at a time: the four index decisions, whose
          // threshold reads are then in flight together, before the four
          // field contributions
#pragma unroll
          for (int cz = 0; cz < 2; ++cz) {
            double r2[4], ri[4], u[4], tn[4];
            int nn[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              r2[q] = exy[q] + z2[cz];  // (dx*dx + dy*dy) + dz*dz
              ri[q] = rsqrt_f64(r2[q]);
              u[q] = __builtin_fma(-(r2[q] * ri[q]), p.inv_cdt, p.a_f);
              nn[q] = (int)__builtin_rint(u[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) tn[q] = thr_at[nn[q]];
            if constexpr (FP) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int mm = r2[q] <= tn[q] ? nn[q] : nn[q] - 1;
                fpa.add(p.a_i + mm, cell_s(s_base, 4 * cz + q));
              }
            } else {
              // the layer's four entries and fractions, then each pair's
              // planes read after the previous pair's fields are formed
              // (fewer registers held across the layer)
              int e[4];
              double fq[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int mm = r2[q] <= tn[q] ? nn[q] : nn[q] - 1;
                e[q] = cellbase + (4 * cz + q) * kCellStride + max(mm, mlo);
                fq[q] = u[q] - (double)mm;
              }
              double P[2][4][4];
              planes_at(lds, PU, e[0], P[0]);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                pair_fields_from<CUB>(P[q & 1], fq[q], ri[q], ex[q & 1], ey[q >> 1], ez[cz], dE, dB, inv_dt);
                if (q < 3) planes_at(lds, PU, e[q + 1], P[(q + 1) & 1]);
              }
            }
          }
          continue;
        }
        const int4 ti = tab[q].i;
        const int lo = ti.x;
        const int hiw = min(ti.y - lo, W - 1);
        const int off = p.a_i - lo;
        const int cellbase = __builtin_amdgcn_readfirstlane(j * kBrickCells * kCellStride + off);
        const int mlo = -off, mhi = hiw - off;
        const double* bc = tab_c[q];
        const int s_base = FP ? brick_s_base(ti.w) : 0;
        const bool fast = (ti.z & 0xff02) == 0xff00;
        const double dx[2] = {rox - bc[0], rox - bc[1]};
        const double dy[2] = {roy - bc[2], roy - bc[3]};
        const double dz[2] = {roz - bc[4], roz - bc[5]};
        const double x2[2] = {dx[0] * dx[0], dx[1] * dx[1]};
        const double y2[2] = {dy[0] * dy[0], dy[1] * dy[1]};
        const double z2[2] = {dz[0] * dz[0], dz[1] * dz[1]};
        const int vmask = ti.z >> 8;
        const bool near = (ti.z & 2) != 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
          if (!fast) {
            if (!((vmask >> c) & 1)) continue;
            if (near && canon_screened(dx[cx], dy[cy], dz[cz], p.screen)) {
              if (FP) fpa.n_scr += 1;
              continue;
            }
          }
          // (dx*dx + dy*dy) + dz*dz, as the canonical sequence
          const double r2 = (x2[cx] + y2[cy]) + z2[cz];
          const double R = __builtin_sqrt(r2);
          const double u = p.a_f - R * p.inv_cdt;
          const double fl = __builtin_floor(u);
          const int mm = (int)__builtin_fmax(fl, -1e9);
          if (FP) {
            fpa.add(p.a_i + mm, cell_s(s_base, c));
            continue;
          }
          const int e = cellbase + c * kCellStride + min(max(mm, mlo), mhi);
          pair_fields<CUB>(lds, PU, e, u - fl, recip_f64(R), dx[cx], dy[cy], dz[cz], dE, dB, inv_dt);
        }
      }
    }
    }
    __syncthreads();
    pos = npos;
    cnt = ncnt;
    more = next;
  }

  if constexpr (sizeof(T) == 4) {
    if (!FP)
      for (int a = 0; a < 3; ++a) {
        two_sum_acc(sE[a], cE[a], bE[a]);
        two_sum_acc(sB[a], cB[a], bB[a]);
      }
  }
  if (!valid) return;
  const long long n_obs = (long long)p.obs.n[0] * p.obs.n[1] * p.obs.n[2];
  const long long o = (long long)ix + (long long)p.obs.n[0] * ((long long)iy + (long long)p.obs.n[1] * iz);
  if (FP) {
    atomicAdd(&p.fp[o * 4 + 0], fpa.n_live);
    atomicAdd(&p.fp[o * 4 + 1], fpa.sum_k);
    atomicAdd(&p.fp[o * 4 + 2], fpa.sum_kw);
    atomicAdd(&p.fp[o * 4 + 3], fpa.n_scr);
    return;
  }
  double tot[6];
  if constexpr (sizeof(T) == 4) {
    for (int a = 0; a < 3; ++a) {
      tot[a] = (double)sE[a] + (double)cE[a];
      tot[3 + a] = (double)sB[a] + (double)cB[a];
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      tot[a] = dE[a];
      tot[3 + a] = dB[a];
    }
  }
  if (p.direct) {
    for (int a = 0; a < 3; ++a) {
      const double e = tot[a] * p.pref, bb = tot[3 + a] * p.pref;
      if (p.out_f64) {
        ((double*)p.E)[a * n_obs + o] = e;
        ((double*)p.B)[a * n_obs + o] = bb;
      } else {
        ((float*)p.E)[a * n_obs + o] = (float)e;
        ((float*)p.B)[a * n_obs + o] = (float)bb;
      }
    }
  } else {
    for (int a = 0; a < 6; ++a) p.partial[((long long)split * 6 + a) * n_obs + o] = tot[a];
  }
}

template <typename T, int WZ, bool FP, int IDX, int W, int STG>
__global__ __launch_bounds__(256 * WZ) __attribute__((amdgpu_waves_per_eu(4))) void pair_kernel_fast(PairParams p) {
  using S = FastShape<T, WZ, W>;
  __shared__ float4 lds[S::NPL * S::PU];
  __shared__ BrickEntry tab[kBrickRing];
  __shared__ double tab_c[kBrickRing][6];
  __shared__ double thr[S::THR];
  __shared__ int qs[2];
  pair_body<T, WZ, FP, IDX, W, STG>(p, xcd_remap((int)blockIdx.x, p.n_wg, p.n_tiles, p.n_splits), lds, tab,
                                    tab_c, thr, qs);
}

// Persistent batched launch: workgroups pull (instance, workgroup id) items
// from a queue ordered heaviest first until it is empty.  IDX as for
// pair_body, one value for the whole batch.
template <typename T, int WZ, int IDX, int STG>
__global__ __launch_bounds__(256 * WZ) __attribute__((amdgpu_waves_per_eu(4))) void pair_kernel_persistent(BatchDevice bd) {
  using S = FastShape<T, WZ, 32>;
  __shared__ float4 lds[S::NPL * S::PU];
  __shared__ BrickEntry tab[kBrickRing];
  __shared__ double tab_c[kBrickRing][6];
  __shared__ double thr[S::THR];
  __shared__ int qs[2];
  __shared__ int cur;
  const int n_items = bd.counts[1 + 2 * bd.group];
  const int2* items = bd.items + bd.counts[2 + 2 * bd.group];
  for (;;) {
    __syncthreads();  // the previous item is done with LDS and `cur`
    if (threadIdx.x == 0) cur = atomicAdd(bd.counter + bd.group, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(cur);
    if (it >= n_items) break;
    const int2 item = items[it];
    const int inst = __builtin_amdgcn_readfirstlane(item.x);
    const int bid = __builtin_amdgcn_readfirstlane(item.y);
    using CP = const __attribute__((address_space(4))) PairParams;
    CP& p = *(CP*)(bd.params + inst);
    pair_body<T, WZ, false, IDX, 32, STG>(p, bid, lds, tab, tab_c, thr, qs);
  }
}

__global__ void threshold_kernel(double* out, int lo, int n, double af, double icdt) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) out[i] = r2_threshold(lo + i, af, icdt);
}

__global__ void batch_threshold(BatchDevice bd) {
  const int n_inst = bd.counts[0];
  for (int inst = (int)blockIdx.y; inst < n_inst; inst += (int)gridDim.y) {
    const PairParams& p = bd.params[inst];
    if (!p.use_thr) continue;
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < p.thr_n; i += (int)(gridDim.x * blockDim.x))
      p.thr[i] = r2_threshold(p.thr_lo + i, p.a_f, p.inv_cdt);
  }
}

__global__ void batch_reset(BatchDevice bd) {
  if (threadIdx.x < 2 && blockIdx.x == 0) bd.counter[threadIdx.x] = 0;
}

// Fixed-order split reduction for every instance of a batch that has splits.
__global__ void batch_epilogue(BatchDevice bd) {
  const int n_inst = bd.counts[0];
  const long long total = bd.epi_prefix[n_inst];
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {  // last instance whose prefix is <= g
      const int mid = (lo + hi + 1) >> 1;
      if (bd.epi_prefix[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const EpilogueParams& ep = bd.epi[lo];
    const long long local = g - bd.epi_prefix[lo];
    const long long comp = local / ep.n_obs;
    const long long o = local - comp * ep.n_obs;
    double s = 0.0;
    for (int q = 0; q < ep.n_splits; ++q) s += ep.partial[((long long)q * 6 + comp) * ep.n_obs + o];
    const double v = s * ep.pref;
    void* dst = comp < 3 ? ep.E : ep.B;
    const long long at = (comp % 3) * ep.n_obs + o;
    if (ep.out_f64)
      ((double*)dst)[at] = v;
    else
      ((float*)dst)[at] = (float)v;
  }
}

__global__ void epilogue_kernel(EpilogueParams p) {
  const long long total = p.n_obs * 6;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long comp = i / p.n_obs;
    const long long o = i - comp * p.n_obs;
    double s = 0.0;
    for (int q = 0; q < p.n_splits; ++q) s += p.partial[((long long)q * 6 + comp) * p.n_obs + o];
    const double v = s * p.pref;
    void* dst = comp < 3 ? p.E : p.B;
    const long long at = (comp % 3) * p.n_obs + o;
    if (p.out_f64)
      ((double*)dst)[at] = v;
    else
      ((float*)dst)[at] = (float)v;
  }
}

__global__ void zero_kernel(uint4* p, unsigned long long n16, unsigned char* tail, int ntail) {
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (unsigned long long)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

template <typename T>
__global__ void ingest_kernel(const T* slice, T* slot, GridD src, int nbx, int nby) {
  const long long n = (long long)src.n[0] * src.n[1] * src.n[2];
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(s % src.n[0]);
    const int j = (int)((s / src.n[0]) % src.n[1]);
    const int k = (int)(s / ((long long)src.n[0] * src.n[1]));
    const long long b = (long long)(i >> 1) + (long long)nbx * ((j >> 1) + (long long)nby * (k >> 1));
    const int c = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
    T* dst = slot + (b * kBrickCells + c) * 4;
    dst[0] = slice[s];
    dst[1] = slice[n + s];
    dst[2] = slice[2 * n + s];
    dst[3] = slice[3 * n + s];
  }
}

// Every slot of a host-layout history [n_slots][4][n] into ring slots of the
// brick layout (blockIdx.y = slot).
template <typename T>
__global__ void ingest_slots_kernel(const T* hist, T* ring, GridD src, int nbx, int nby, long long slot_elems) {
  const long long n = (long long)src.n[0] * src.n[1] * src.n[2];
  const T* slice = hist + (long long)blockIdx.y * 4 * n;
  T* slot = ring + (long long)blockIdx.y * slot_elems;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(s % src.n[0]);
    const int j = (int)((s / src.n[0]) % src.n[1]);
    const int k = (int)(s / ((long long)src.n[0] * src.n[1]));
    const long long b = (long long)(i >> 1) + (long long)nbx * ((j >> 1) + (long long)nby * (k >> 1));
    const int c = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
    T* dst = slot + (b * kBrickCells + c) * 4;
    dst[0] = slice[s];
    dst[1] = slice[n + s];
    dst[2] = slice[2 * n + s];
    dst[3] = slice[3 * n + s];
  }
}

__global__ void fill_zero_fields(void* E, void* B, long long n, int f64) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n;
       i += (long long)gridDim.x * blockDim.x) {
    if (f64) {
      ((double*)E)[i] = 0.0;
      ((double*)B)[i] = 0.0;
    } else {
      ((float*)E)[i] = 0.f;
      ((float*)B)[i] = 0.f;
    }
  }
}

// One thread per (observation point, source cell): the slice decision taken
// by the pair kernels, from the same coordinate construction (tile reference
// point, brick corner, cell offset) and the same index code.
__global__ void dump_kernel(DumpParams p) {
  const long long ns = (long long)p.src.n[0] * p.src.n[1] * p.src.n[2];
  const long long no = (long long)p.obs.n[0] * p.obs.n[1] * p.obs.n[2];
  const long long total = ns * no;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const long long o = q / ns;
    const long long s = q - o * ns;
    const int ix = (int)(o % p.obs.n[0]);
    const int iy = (int)((o / p.obs.n[0]) % p.obs.n[1]);
    const int iz = (int)(o / ((long long)p.obs.n[0] * p.obs.n[1]));
    const int si = (int)(s % p.src.n[0]);
    const int sj = (int)((s / p.src.n[0]) % p.src.n[1]);
    const int sk = (int)(s / ((long long)p.src.n[0] * p.src.n[1]));
    const double rox = canon(p.obs.o[0], ix, p.obs.h[0]);
    const double roy = canon(p.obs.o[1], iy, p.obs.h[1]);
    const double roz = canon(p.obs.o[2], iz, p.obs.h[2]);
    const double rsx = canon(p.src.o[0], si, p.src.h[0]);
    const double rsy = canon(p.src.o[1], sj, p.src.h[1]);
    const double rsz = canon(p.src.o[2], sk, p.src.h[2]);
    int code;
    if (canon_screened(rox - rsx, roy - rsy, roz - rsz, p.screen)) {
      code = INT32_MIN;
    } else {
      int k;
      if (p.use_f64) {
        const double u = canon_u(rox - rsx, roy - rsy, roz - rsz, p.a_f, p.inv_cdt);
        k = p.a_i + (int)__builtin_fmax(__builtin_floor(u), -1e9);
      } else {
        const int tx0 = (ix / kTileEdge) * kTileEdge, ty0 = (iy / kTileEdge) * kTileEdge,
                  tz0 = (iz / kTileEdge) * kTileEdge;
        const double refx = canon(p.obs.o[0], tx0, p.obs.h[0]);
        const double refy = canon(p.obs.o[1], ty0, p.obs.h[1]);
        const double refz = canon(p.obs.o[2], tz0, p.obs.h[2]);
        const double ls = p.inv_cdt;
        const float xo = (float)((rox - refx) * ls), yo = (float)((roy - refy) * ls),
                    zo = (float)((roz - refz) * ls);
        const double bxc = canon(p.src.o[0], si & ~1, p.src.h[0]);
        const double byc = canon(p.src.o[1], sj & ~1, p.src.h[1]);
        const double bzc = canon(p.src.o[2], sk & ~1, p.src.h[2]);
        const float d0x = xo - (float)((bxc - refx) * ls);
        const float d0y = yo - (float)((byc - refy) * ls);
        const float d0z = zo - (float)((bzc - refz) * ls);
        const float dx = (si & 1) ? d0x - (float)(p.src.h[0] * ls) : d0x;
        const float dy = (sj & 1) ? d0y - (float)(p.src.h[1] * ls) : d0y;
        const float dz = (sk & 1) ? d0z - (float)(p.src.h[2] * ls) : d0z;
        float m, f, ri;
        index_f32(dx, dy, dz, (float)p.a_f, 0.5f - p.guard,
                  [&]() { return canon_u(rox - rsx, roy - rsy, roz - rsz, p.a_f, p.inv_cdt); }, m, f,
                  ri);
        k = p.a_i + (int)m;
      }
      code = k < -1 ? -2 : k;
    }
    p.out[q] = code;
  }
}

int grid_for(long long n, int block) {
  long long g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_zero(void* p, unsigned long long bytes, hipStream_t s) {
  const unsigned long long n16 = bytes / 16;
  const int ntail = (int)(bytes - n16 * 16);
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for((long long)(n16 > 0 ? n16 : 1), 256)), dim3(256), 0, s,
                     (uint4*)p, n16, (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError();
}

hipError_t launch_ingest(const void* slice, void* slot, const GridD& src, int nbx, int nby,
                         int is_f64, hipStream_t s) {
  const long long n = (long long)src.n[0] * src.n[1] * src.n[2];
  if (n == 0) return hipSuccess;
  if (is_f64)
    hipLaunchKernelGGL(ingest_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       (const double*)slice, (double*)slot, src, nbx, nby);
  else
    hipLaunchKernelGGL(ingest_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       (const float*)slice, (float*)slot, src, nbx, nby);
  return hipGetLastError();
}

hipError_t launch_ingest_slots(const void* hist, void* ring, const GridD& src, int nbx, int nby, int n_slots,
                               int is_f64, hipStream_t s) {
  const long long n = (long long)src.n[0] * src.n[1] * src.n[2];
  if (n == 0 || n_slots <= 0) return hipSuccess;
  const long long nb = (long long)nbx * nby * (((long long)src.n[2] + 1) / 2);
  const long long slot_elems = nb * kBrickCells * 4;
  const size_t esz = is_f64 ? 8 : 4;
  for (int first = 0; first < n_slots; first += 65535) {
    const int cnt = std::min(65535, n_slots - first);
    const dim3 grid((unsigned)std::min<long long>(grid_for(n, 256), 1024), (unsigned)cnt);
    const char* h = (const char*)hist + (size_t)first * 4 * (size_t)n * esz;
    char* r = (char*)ring + (size_t)first * (size_t)slot_elems * esz;
    if (is_f64)
      hipLaunchKernelGGL(ingest_slots_kernel<double>, grid, dim3(256), 0, s, (const double*)h, (double*)r, src,
                         nbx, nby, slot_elems);
    else
      hipLaunchKernelGGL(ingest_slots_kernel<float>, grid, dim3(256), 0, s, (const float*)h, (float*)r, src, nbx,
                         nby, slot_elems);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pairs(const PairParams& p, int is_f64, int fingerprint, int multi_chunk, int wsel,
                        hipStream_t s) {
  dim3 grid(p.n_wg), block(kThreads);
  // the fingerprint pass takes slice decisions only: no staging variants
  const bool cub = !fingerprint && (p.stencil & kStencilCubic) != 0;
  const bool cut = !fingerprint && (p.stencil & kStencilCut) != 0;
#define JEFI_LAUNCH(T, G, FPM, MUL) \
  hipLaunchKernelGGL((pair_kernel<T, G, FPM, MUL>), grid, block, 0, s, p)
#define JEFI_FAST(T, WZ, FPM, IDX, W)                                                                    \
  do {                                                                                                  \
    if (FPM)                                                                                            \
      hipLaunchKernelGGL((pair_kernel_fast<T, WZ, true, IDX, W, 0>), grid, dim3(256 * WZ), 0, s, p);    \
    else if (cub && cut)                                                                                \
      hipLaunchKernelGGL((pair_kernel_fast<T, WZ, false, IDX, W, 3>), grid, dim3(256 * WZ), 0, s, p);   \
    else if (cub)                                                                                       \
      hipLaunchKernelGGL((pair_kernel_fast<T, WZ, false, IDX, W, 1>), grid, dim3(256 * WZ), 0, s, p);   \
    else if (cut)                                                                                       \
      hipLaunchKernelGGL((pair_kernel_fast<T, WZ, false, IDX, W, 2>), grid, dim3(256 * WZ), 0, s, p);   \
    else                                                                                                \
      hipLaunchKernelGGL((pair_kernel_fast<T, WZ, false, IDX, W, 0>), grid, dim3(256 * WZ), 0, s, p);   \
  } while (0)
#define JEFI_FAST_F32(WZ, FPM, W)        \
  do {                                  \
    if (p.exact_idx)                    \
      JEFI_FAST(float, WZ, FPM, 1, W);  \
    else                                \
      JEFI_FAST(float, WZ, FPM, 0, W);  \
  } while (0)
  if (!multi_chunk && wsel > 32) {
    // long windows: 8x8x8 tiles, fewer bricks per round
    if (is_f64) {
      if (fingerprint) JEFI_FAST(double, 2, true, 0, 64); else JEFI_FAST(double, 2, false, 0, 64);
    } else if (wsel == 64) {
      if (fingerprint) JEFI_FAST_F32(2, true, 64); else JEFI_FAST_F32(2, false, 64);
    } else {
      if (fingerprint) JEFI_FAST_F32(2, true, 128); else JEFI_FAST_F32(2, false, 128);
    }
    return hipGetLastError();
  }
  if (!multi_chunk) {
    if (p.tile_z == 8) {
      if (is_f64) {
        if (fingerprint) JEFI_FAST(double, 2, true, 0, 32); else JEFI_FAST(double, 2, false, 0, 32);
      } else {
        if (fingerprint) JEFI_FAST_F32(2, true, 32); else JEFI_FAST_F32(2, false, 32);
      }
    } else {
      if (is_f64) {
        if (fingerprint) JEFI_FAST(double, 1, true, 0, 32); else JEFI_FAST(double, 1, false, 0, 32);
      } else {
        if (fingerprint) JEFI_FAST_F32(1, true, 32); else JEFI_FAST_F32(1, false, 32);
      }
    }
    return hipGetLastError();
  }
  if (is_f64) {
    if (fingerprint) {
      if (multi_chunk) JEFI_LAUNCH(double, 2, true, true); else JEFI_LAUNCH(double, 2, true, false);
    } else {
      if (multi_chunk) JEFI_LAUNCH(double, 2, false, true); else JEFI_LAUNCH(double, 2, false, false);
    }
  } else {
    if (fingerprint) {
      if (multi_chunk) JEFI_LAUNCH(float, 4, true, true); else JEFI_LAUNCH(float, 4, true, false);
    } else {
      if (multi_chunk) JEFI_LAUNCH(float, 4, false, true); else JEFI_LAUNCH(float, 4, false, false);
    }
  }
#undef JEFI_LAUNCH
#undef JEFI_FAST
  return hipGetLastError();
}

hipError_t launch_thresholds(double* out, int lo, int n, double af, double icdt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(threshold_kernel, dim3((n + 127) / 128), dim3(128), 0, s, out, lo, n, af, icdt);
  return hipGetLastError();
}

void* batch_reset_kernel() { return (void*)batch_reset; }
void* batch_threshold_kernel() { return (void*)batch_threshold; }
void* batch_epilogue_kernel() { return (void*)batch_epilogue; }
template <int STG>
static void* batch_pair_kernel_stg(int is_f64, int wz, int idx) {
  if (is_f64)
    return wz == 2 ? (void*)pair_kernel_persistent<double, 2, 0, STG> : (void*)pair_kernel_persistent<double, 1, 0, STG>;
  if (idx)
    return wz == 2 ? (void*)pair_kernel_persistent<float, 2, 1, STG> : (void*)pair_kernel_persistent<float, 1, 1, STG>;
  return wz == 2 ? (void*)pair_kernel_persistent<float, 2, 0, STG> : (void*)pair_kernel_persistent<float, 1, 0, STG>;
}

void* batch_pair_kernel(int is_f64, int wz, int idx, int stg) {
  switch (stg) {
    case 1: return batch_pair_kernel_stg<1>(is_f64, wz, idx);
    case 2: return batch_pair_kernel_stg<2>(is_f64, wz, idx);
    case 3: return batch_pair_kernel_stg<3>(is_f64, wz, idx);
    default: return batch_pair_kernel_stg<0>(is_f64, wz, idx);
  }
}
int batch_pair_threads(int wz) { return 256 * wz; }

hipError_t launch_epilogue(const EpilogueParams& p, hipStream_t s) {
  if (p.n_obs == 0) return hipSuccess;
  hipLaunchKernelGGL(epilogue_kernel, dim3(grid_for(p.n_obs * 6, 256)), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_fill_zero_fields(void* E, void* B, long long n_obs, int out_f64, hipStream_t s) {
  if (n_obs == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_fields, dim3(grid_for(3 * n_obs, 256)), dim3(256), 0, s, E, B, n_obs,
                     out_f64);
  return hipGetLastError();
}

hipError_t launch_dump(const DumpParams& p, hipStream_t s) {
  const long long ns = (long long)p.src.n[0] * p.src.n[1] * p.src.n[2];
  const long long no = (long long)p.obs.n[0] * p.obs.n[1] * p.obs.n[2];
  if (ns * no == 0) return hipSuccess;
  hipLaunchKernelGGL(dump_kernel, dim3(grid_for(ns * no, 256)), dim3(256), 0, s, p);
  return hipGetLastError();
}

// Scratch of the allocation-free evaluation: one fixed array per GPU, held
// until the process ends.  Host code never uses the array's name as an
// address: each device's copy is looked up once, with that device current,
// and that address is what kernels receive.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** out) {
  static std::mutex mu;
  static std::map<int, void*> by_device;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = by_device.find(dev);
  if (it == by_device.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (ptr == nullptr) return hipErrorInvalidSymbol;
    it = by_device.emplace(dev, ptr).first;
  }
  *out = it->second;
  return hipSuccess;
}

}  // namespace jefi
