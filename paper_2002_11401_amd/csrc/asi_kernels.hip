// HIP kernels (gfx950) of the spin-ice relaxation path.
//
// Model: flatspin dipole model (Jensen et al.), Sec. II.  All field and
// margin arithmetic is FP64 and this file is compiled without FMA
// contraction, so every kernel that evaluates the same expression on the
// same inputs produces the same bits -- plain, batched and served runs agree
// bitwise by construction.
//
//   k_nb_count / k_nb_fill  neighbour tables of Sec. II.C and the projected
//                           couplings of Eq. 3 (once per instance)
//   k_field                 full-field pass: Eq. 3 gathered in ascending
//                           neighbour order, plus applied field (Sec. II.D)
//                           and thermal field (Sec. II.E), Eq. 2, projected;
//                           switching key of Eq. 5 / Eq. 6; per-64-row maxima
//   k_relax                 one workgroup per instance: argmax over the
//                           flippable keys (ties: lowest index), flip, update
//                           the neighbours' fields incrementally, repeat
//                           until none can flip (Sec. II.H)
//   k_fused                 one workgroup per instance runs whole steps
//                           (field phase + relax) through its own protocol
#include <algorithm>
#include <climits>
#include <mutex>

#define ASI_KERNELS_UNIT 1
#include "asi_internal.h"

namespace asi {
namespace {

// ------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds; each round
// multiplies counter words 0 and 2 by the two round multipliers and xors the
// high halves into words 1 and 3 with the key; the key advances by the two
// Weyl increments between rounds.
struct U4 {
  uint32_t x, y, z, w;
};

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// Thermal field of Sec. II.E: two independent N(0,1) draws for magnet i at
// step t (counter (i, t, 0, 0)), by Box-Muller on 53-bit uniforms
// u1 in (0, 1] and u2 in [0, 1).
__device__ inline void thermal_normals(uint64_t seed, uint32_t i, uint32_t t, double& z0,
                                       double& z1) {
  const U4 o = philox4x32_10(U4{i, t, 0u, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((((uint64_t)o.x) << 32) | o.y) >> 11;
  const uint64_t b = ((((uint64_t)o.z) << 32) | o.w) >> 11;
  const double u1 = (double)(a + 1) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  double sn, cs;
  sincos(ang, &sn, &cs);
  z0 = rad * cs;
  z1 = rad * sn;
}

// Upper bound of x^e (x >= 0, e > 0) from the single-precision hardware
// log2 and exp2, inflated by 0.1 %, far past their error (a few units in
// the 24th bit of the exponent and of the result); x below 2^-100 is raised
// to 2^-100, which only raises x^e.
__device__ inline float pow_bound(double x, double e) {
  const float xf = (float)fmax(x, 0x1p-100);
  return __builtin_amdgcn_exp2f((float)e * __builtin_amdgcn_logf(xf)) * 1.001f;
}

// Switching key: the left-hand side of Eq. 5 when magnet i may flip, i.e.
// the field opposes the moment (Eq. 6, s_i h_par < 0) and Eq. 5 exceeds 1;
// otherwise 0.  Exponents ep = 2/gamma, eq = 2/beta.  When the bound puts
// the left-hand side below 1 the FP64 powers (which could only give a
// value <= 1: the bound exceeds their sum) are skipped: the key is the
// same, bit for bit.
// In two stages: key_needs_powers settles the key at 0, or gives the
// normalised field components a and q whose powers decide it.
__device__ inline bool key_needs_powers(int s, double hp, double hq, double hk, double b,
                                        double c, double ep, double eq, double& a, double& q) {
  // h_k > 0 always (checked at creation); testing it with the direction
  // makes h_k needed on every path, so its load is issued with the field's
  // and the spin's instead of after them
  const bool against = (hk > 0.0) && ((s > 0) ? (hp < 0.0) : (hp > 0.0));
  if (!against) return false;
  a = fabs(hp) / (b * hk);
  q = fabs(hq) / (c * hk);
  return !(pow_bound(a, ep) + pow_bound(q, eq) < 1.0f);
}
__device__ inline double key_from_powers(double a, double q, double ep, double eq) {
  const double L = pow(a, ep) + pow(q, eq);
  return (L > 1.0) ? L : 0.0;
}
__device__ inline double switching_key(int s, double hp, double hq, double hk, double b,
                                       double c, double ep, double eq) {
  double a = 0.0, q = 0.0;
  if (!key_needs_powers(s, hp, hq, hk, b, c, ep, eq, a, q)) return 0.0;
  return key_from_powers(a, q, ep, eq);
}

// Eq. 3 for a unit source moment mhat_s at (sx, sy) seen at (fx, fy),
// projected on the observer's easy axis (A) and hard axis (B);
// mhatperp = (-my, mx).  A is symmetric in (f, s) bit for bit: swapping
// the two negates r, which negates both dot products of the 3(.)(.) term.
__device__ inline void coupling(double fx, double fy, double fmx, double fmy, double sx,
                                double sy, double smx, double smy, double alpha, double& A,
                                double& B) {
  const double rx = fx - sx;
  const double ry = fy - sy;
  const double r2 = rx * rx + ry * ry;
  const double r = sqrt(r2);
  const double inv3 = 1.0 / (r2 * r);
  const double inv5 = inv3 / r2;
  const double af = fmx * rx + fmy * ry;
  const double as = smx * rx + smy * ry;
  const double pf = fmx * ry - fmy * rx;
  const double mm = fmx * smx + fmy * smy;
  const double pm = fmx * smy - fmy * smx;
  A = alpha * (3.0 * (af * as) * inv5 - mm * inv3);
  B = alpha * (3.0 * (pf * as) * inv5 - pm * inv3);
}

// Cross-lane moves of a double within rows of 16 lanes by DPP.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ inline double readlane_f64(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Maximum over the 64 lanes, returned to every lane: butterfly within each
// row of 16 (quad swaps, half-row and row mirrors), then the four row
// results through scalar reads.
__device__ inline double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x141>(v));  // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));  // row_mirror
  const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
  const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
  return fmax(fmax(r0, r1), fmax(r2, r3));
}

// Wave-wide argmax of (key, payload) where lane order is index order:
// largest key, and among equal keys the lowest lane.  All 64 lanes call;
// the result is uniform.
__device__ inline void wave_argmax(double& key, uint32_t& payload) {
  const double m = wave_max_f64(key);
  const unsigned long long bal = __ballot(key == m);
  const int src = __ffsll((unsigned long long)bal) - 1;
  payload = (uint32_t)__builtin_amdgcn_readlane((int)payload, src);
  key = m;
}

__device__ inline int64_t slot_of(int64_t i, int32_t D, int32_t k) {
  return ((i >> 6) * (int64_t)D + k) * kSlice + (i & (kSlice - 1));
}

// ------------------------------------------------------------ neighbours
// Coercive fields of Sec. II.G drawn on the device (hk == NULL): the first
// Box-Muller normal of Philox4x32-10 at counter (i, 0, 1, 0), uniforms
// formed as for the thermal field.
__global__ void k_draw_hk(double* __restrict__ hk, int64_t n, double mean, double k,
                          uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const U4 o = philox4x32_10(U4{(uint32_t)i, 0u, 1u, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((((uint64_t)o.x) << 32) | o.y) >> 11;
  const uint64_t b = ((((uint64_t)o.z) << 32) | o.w) >> 11;
  const double u1 = (double)(a + 1) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  const double z0 = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  const double sd = k * mean;
  const double h = mean + sd * z0;
  const double lo = 1e-12 * mean;
  hk[i] = h < lo ? lo : h;
}

// Cells of side >= the cutoff, magnets sorted by cell (ascending index
// within a cell); a magnet's neighbours lie in its 3 x 3 cell block.
__global__ void k_nb_count(const double* __restrict__ x, const double* __restrict__ y,
                           const int32_t* __restrict__ cellx, const int32_t* __restrict__ celly,
                           const int32_t* __restrict__ cstart, const int32_t* __restrict__ cmem,
                           int64_t n, int64_t gx, int64_t gy, double cut2,
                           int32_t* __restrict__ len, int32_t* __restrict__ dup) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i];
  const int64_t cx = cellx[i], cy = celly[i];
  int32_t cnt = 0;
  for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
    if (yy < 0 || yy >= gy) continue;
    for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
      if (xx < 0 || xx >= gx) continue;
      const int64_t c = yy * gx + xx;
      for (int32_t p = cstart[c]; p < cstart[c + 1]; ++p) {
        const int32_t j = cmem[p];
        if (j == i) continue;
        const double dx = xi - x[j];
        const double dy = yi - y[j];
        const double r2 = dx * dx + dy * dy;
        if (r2 <= cut2) {
          ++cnt;
          if (r2 == 0.0) *dup = 1;
        }
      }
    }
  }
  len[i] = cnt;
}

// Fills row i in ascending neighbour order by a 9-way merge of the
// (ascending) member lists of its 3 x 3 cell block, and computes the
// projected couplings of each pair; writes the sliced and the row-major
// tables.
__global__ void k_nb_fill(const double* __restrict__ x, const double* __restrict__ y,
                          const double* __restrict__ mx, const double* __restrict__ my,
                          const int32_t* __restrict__ cellx, const int32_t* __restrict__ celly,
                          const int32_t* __restrict__ cstart, const int32_t* __restrict__ cmem,
                          int64_t n, int64_t gx, int64_t gy, double cut2, double alpha,
                          int32_t D, int32_t* __restrict__ col, double* __restrict__ A,
                          double* __restrict__ B, int32_t* __restrict__ rcol,
                          double* __restrict__ rA, double* __restrict__ rBr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i], mxi = mx[i], myi = my[i];
  const int64_t cx = cellx[i], cy = celly[i];
  int32_t pos[9], end[9], head[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int64_t xx = cx + (r % 3) - 1;
    const int64_t yy = cy + (r / 3) - 1;
    const bool ok = xx >= 0 && xx < gx && yy >= 0 && yy < gy;
    const int64_t c = yy * gx + xx;
    pos[r] = ok ? cstart[c] : 0;
    end[r] = ok ? cstart[c + 1] : 0;
    head[r] = pos[r] < end[r] ? cmem[pos[r]] : INT_MAX;
  }
  int32_t k = 0;
  while (true) {
    int32_t best = INT_MAX;
    int br = -1;
#pragma unroll
    for (int r = 0; r < 9; ++r)
      if (head[r] < best) {
        best = head[r];
        br = r;
      }
    if (br < 0) break;
#pragma unroll
    for (int r = 0; r < 9; ++r)
      if (r == br) {
        ++pos[r];
        head[r] = pos[r] < end[r] ? cmem[pos[r]] : INT_MAX;
      }
    const int32_t j = best;
    if (j == i) continue;
    const double xj = x[j], yj = y[j];
    const double dx = xi - xj;
    const double dy = yi - yj;
    if (dx * dx + dy * dy > cut2) continue;
    if (k >= D) break;  // cannot happen: D is the maximum count
    double a, b, ar, bt;
    const double mxj = mx[j], myj = my[j];
    coupling(xi, yi, mxi, myi, xj, yj, mxj, myj, alpha, a, b);
    coupling(xj, yj, mxj, myj, xi, yi, mxi, myi, alpha, ar, bt);
    const int64_t sl = slot_of(i, D, k);
    col[sl] = j;
    A[sl] = a;
    B[sl] = b;
    const int64_t rs = i * D + k;
    rcol[rs] = j;
    rA[rs] = a;
    rBr[rs] = bt;
    ++k;
  }
  for (; k < D; ++k) {
    const int64_t sl = slot_of(i, D, k);
    col[sl] = -1;
    A[sl] = 0.0;
    B[sl] = 0.0;
    const int64_t rs = i * D + k;
    rcol[rs] = -1;
    rA[rs] = 0.0;
    rBr[rs] = 0.0;
  }
}

// ------------------------------------------------------------ field phase
// Field of row i at step t (Eq. 2): the dipolar sum of Eq. 3 -- gathered over
// the neighbours in ascending order with one accumulator per axis, left to
// right, or carried from earlier steps -- plus H[t], any local external
// field and the thermal draw, projected on the easy and hard axis; then the
// switching key.  Writes the row's total field and key and returns (key,
// index | sign bit).  Every field pass (grid-wide or inside a fused
// workgroup) calls this one function, so they agree bit for bit.
__device__ __forceinline__ double field_finish(const InstDev* __restrict__ I, int64_t i, int64_t t,
                                               double p, double pq, uint32_t& payload);

// Slots per chunk of the canonical dipolar sum (and of the high-degree
// pass), and entries per thread per chunk in the high-degree pass.
constexpr int kHdChunk = 64;
constexpr int kHdPer = 8;

__device__ __forceinline__ double field_row(const InstDev* __restrict__ I, int64_t i, int64_t t,
                                   uint32_t& payload) {
  const int8_t* __restrict__ s = I->s;
  const int32_t mode = I->field_mode;
  double p, pq;
  if (mode == kFieldFull || I->dirty[i]) {
    const int32_t L = I->len[i];
    const int64_t base = slot_of(i, I->D, 0);
    const int32_t* __restrict__ col = I->col + base;
    const double* __restrict__ A = I->A + base;
    const double* __restrict__ B = I->B + base;
    // Groups of 8 neighbours; the columns of the next group are fetched
    // with the couplings and spins of the current one, so each group costs
    // one round trip.  The canonical order of the sum: each chunk of 64
    // slots is added in ascending order from zero, and the chunk sums in
    // ascending order (up to 64 neighbours, the plain left-to-right sum);
    // every pass uses it, so all agree bit for bit.  The tables are streamed
    // once per pass (non-temporal loads), which leaves the L2 to the
    // gathered spins.
    // (A chunk sum that ends on a 64-slot boundary is added there, the last
    // one after the loop; a zero added after a full last chunk is exact.)
    p = 0.0;
    pq = 0.0;
    double cp = 0.0, cq = 0.0;
    int32_t jc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) jc[u] = (u < L) ? __builtin_nontemporal_load(&col[u * kSlice]) : 0;
    for (int32_t k = 0; k < L; k += 8) {
      double a[8], b[8];
      int sg[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = k + u < L;
        a[u] = ok ? __builtin_nontemporal_load(&A[(k + u) * kSlice]) : 0.0;
        b[u] = ok ? __builtin_nontemporal_load(&B[(k + u) * kSlice]) : 0.0;
        sg[u] = ok ? s[jc[u]] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) jc[u] = (k + 8 + u < L) ? __builtin_nontemporal_load(&col[(k + 8 + u) * kSlice]) : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (k + u < L) {
          cp += (sg[u] > 0) ? a[u] : -a[u];
          cq += (sg[u] > 0) ? b[u] : -b[u];
        }
      }
      if (((k + 8) & (kHdChunk - 1)) == 0) {
        p += cp;
        pq += cq;
        cp = 0.0;
        cq = 0.0;
      }
    }
    p += cp;
    pq += cq;
    if (mode != kFieldFull) {
      I->hd[i] = make_double2(p, pq);
      I->dirty[i] = 0;
    }
  } else {
    // carried, or no neighbour flipped since the last gather
    const double2 c = I->hd[i];
    p = c.x;
    pq = c.y;
  }
  return field_finish(I, i, t, p, pq, payload);
}

// Eq. 2 for row i from its dipolar sums (p, pq): plus H[t], the magnet's
// local external field (if any) and the thermal draw, projected; writes the total field and the key, returns the key.
__device__ __forceinline__ double field_finish(const InstDev* __restrict__ I, int64_t i, int64_t t,
                                               double p, double pq, uint32_t& payload) {
  const int8_t* __restrict__ s = I->s;
  const double mxi = I->mx[i], myi = I->my[i];
  double hp = p, hq = pq;
  if (t >= 0) {
    const double Hx = I->H[2 * t], Hy = I->H[2 * t + 1];
    hp = hp + (Hx * mxi + Hy * myi);
    hq = hq + (Hy * mxi - Hx * myi);
    if (I->hloc) {
      // the magnet's own external field (Sec. II.D), static or of step t
      const double2 l = I->hloc[(I->hloc_k > 1 ? t * I->n : 0) + i];
      hp = hp + (l.x * mxi + l.y * myi);
      hq = hq + (l.y * mxi - l.x * myi);
    }
    if (I->wave_ph) {
      // a travelling wave (Sec. II.D), evaluated here instead of stored per step
      const double a = I->wave_amp * sin(I->wave_ph[i] - I->wave_w * (double)t);
      const double lx = a * I->wave_ex, ly = a * I->wave_ey;
      hp = hp + (lx * mxi + ly * myi);
      hq = hq + (ly * mxi - lx * myi);
    }
    const double sg = I->sigma_t ? I->sigma_t[t] : I->sigma;
    if (sg > 0.0) {
      double z0, z1;
      thermal_normals(I->seed, (uint32_t)i, (uint32_t)t, z0, z1);
      const double tx = sg * z0, ty = sg * z1;
      hp = hp + (tx * mxi + ty * myi);
      hq = hq + (ty * mxi - tx * myi);
    }
  }
  I->h[i] = make_double2(hp, hq);
  const int si = s[i];
  const double key = switching_key(si, hp, hq, I->hk[i], I->b, I->c, I->e_par, I->e_perp);
  I->key[i] = key;
  payload = (uint32_t)i | (si < 0 ? 0x80000000u : 0u);
  return key;
}

// Key of row i as the state holds it, for an instance whose relax paused
// mid-step: the relax keeps every key exact, so its candidate structures
// are rebuilt from the key array instead of a field evaluation.
__device__ __forceinline__ double stored_key(const InstDev* __restrict__ I, int64_t i,
                                             uint32_t& payload) {
  payload = (uint32_t)i | (I->s[i] < 0 ? 0x80000000u : 0u);
  return I->key[i];
}

// Field phase for the 64 rows starting at row0 (a multiple of 64), by one
// wavefront: rows (or, resuming a paused relax, their stored keys), then
// their maximum key into the per-64-row table.  Returns the lane's (key,
// payload) for the candidate pool.
__device__ __forceinline__ double field_rows64(const InstDev* __restrict__ I, int64_t row0,
                                               int64_t t, uint32_t& payload,
                                               bool resume = false) {
  const int lane = threadIdx.x & 63;
  const int64_t i = row0 + lane;
  double key = 0.0;
  payload = 0;
  if (i < I->n) key = resume ? stored_key(I, i, payload) : field_row(I, i, t, payload);
  double mk = key;
  uint32_t mp = payload;
  wave_argmax(mk, mp);
  if (lane == 0) {
    I->t1key[row0 >> 6] = mk;
    I->t1idx[row0 >> 6] = mp;
  }
  return key;
}

// Append a flippable lane's entry at pool position base + its rank among
// the flippable lanes of the wavefront.
__device__ __forceinline__ void pool_put(const InstDev* __restrict__ I, double key,
                                         uint32_t payload, unsigned long long bal, int64_t base) {
  const int lane = threadIdx.x & 63;
  if (key > 0.0) {
    const int64_t q = base + __popcll(bal & ((1ull << lane) - 1ull));
    // A pass appends each row at most once to a pool emptied before it, so
    // q < n < ccap; past the end the entry is dropped and the relax, which
    // finds the count above ccap, fails the step (kPoolOverflow).
    if (q >= I->ccap) return;
    const uint32_t i = payload & 0x7fffffffu;
    I->cpay[0][q] = payload;
    I->ckey[0][q] = key;
    I->cver[0][q] = I->ver[i];
  }
}

// Field phase by one wavefront, appending its flippable rows to the pool
// with one atomic per wavefront.
__device__ __forceinline__ void field_rows64_pool(const InstDev* __restrict__ I, int64_t row0,
                                                  int64_t t, bool resume = false) {
  uint32_t payload;
  const double key = field_rows64(I, row0, t, payload, resume);
  const unsigned long long bal = __ballot(key > 0.0);
  if (bal) {
    int base = 0;
    if ((threadIdx.x & 63) == 0) base = atomicAdd(I->ccount, __popcll(bal));
    base = __builtin_amdgcn_readfirstlane(base);
    pool_put(I, key, payload, bal, base);
  }
}

// Grid-wide field pass: one lane per magnet, any number of instances; the
// block's flippable rows reach the pool with one atomic per block.  A paused
// instance (see RunDev) gets its relax structures rebuilt instead.
__global__ __launch_bounds__(kFieldBlock) void k_field(const InstDev* __restrict__ insts,
                                                      RunDev* __restrict__ runs,
                                                      const int32_t* __restrict__ blk_inst,
                                                      const int32_t* __restrict__ blk_row0) {
  __shared__ int wcount[kFieldBlock / 64];
  __shared__ int bbase;
  const int q = blk_inst[blockIdx.x];
  const RunDev* R = runs + q;
  const bool resume = R->paused != 0;
  if (!R->active && !resume) return;
  const InstDev* I = insts + q;
  const int wave = threadIdx.x >> 6;
  const int64_t wave_row0 = (int64_t)blk_row0[blockIdx.x] + wave * 64;
  uint32_t payload = 0;
  double key = 0.0;
  if (wave_row0 < I->n) key = field_rows64(I, wave_row0, R->t, payload, resume);
  const unsigned long long bal = __ballot(key > 0.0);
  if ((threadIdx.x & 63) == 0) wcount[wave] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < kFieldBlock / 64; ++w) {
      const int c = wcount[w];
      wcount[w] = tot;
      tot += c;
    }
    bbase = tot ? atomicAdd(I->ccount, tot) : 0;
  }
  __syncthreads();
  if (bal) pool_put(I, key, payload, bal, (int64_t)bbase + wcount[wave]);
}

// Full-field pass for an instance of high degree (every row gathered): a
// workgroup of 8 R threads takes R consecutive rows of a 64-row slice (R =
// 64, 32, 16 or 8, fewer rows per workgroup for smaller instances, so that
// the device holds enough workgroups).  Each thread keeps one row, so it
// loads only that row's real slots (slot < len): no padding is read.  The
// slots are read in chunks of kHdChunk, eight entries per thread, the next
// chunk's couplings and spins in flight while the current one is added and
// the columns two chunks ahead; each entry's signed couplings are staged in
// LDS, and the lane of each row adds its chunk in ascending slot order: the
// same sums, in the same order, as field_row.  The workgroups of one slice
// are launched on the same XCD (block ids that differ by multiples of 8),
// so lines shared by two of them are fetched into one L2.

template <int R>
__global__ __launch_bounds__(8 * R) void k_field_hd(const InstDev* __restrict__ insts,
                                                    RunDev* __restrict__ runs) {
  constexpr int S = 64 / R;  // workgroups per slice
  __shared__ double sa[kHdChunk * R];
  __shared__ double sb[kHdChunk * R];
  __shared__ int lmax;
  const RunDev* Rn = runs;
  if (!Rn->active) return;
  const InstDev* I = insts;
  const int q = blockIdx.x;
  const int64_t slice = (int64_t)(q / (8 * S)) * 8 + (q % 8);
  const int sub = (q / 8) % S;
  const int64_t row0 = slice * 64;
  if (row0 >= I->n) return;
  const int tid = threadIdx.x;
  const int r = tid % R;    // the thread's row in the workgroup's R rows
  const int s0 = tid / R;   // its first slot in a chunk; then every 8th
  const int64_t i = row0 + sub * R + r;
  const int32_t L = (i < I->n) ? I->len[i] : 0;
  const int32_t D = I->D;
  const int64_t base = slot_of(row0, D, 0) + sub * R + r;  // slot 0 of the thread's row
  const int8_t* __restrict__ s = I->s;
  if (tid == 0) lmax = 0;
  __syncthreads();
  if (tid < R && L > 0) atomicMax(&lmax, L);
  __syncthreads();
  const int32_t Lw = lmax;  // slots of the longest of the workgroup's rows
  double p = 0.0, pq = 0.0;
  int32_t jc[kHdPer];
  double a[kHdPer], b[kHdPer];
  int sg[kHdPer];
  // chunk 0: columns, then couplings and spins; columns of chunk 1
#pragma unroll
  for (int u = 0; u < kHdPer; ++u) {
    const int k = s0 + 8 * u;
    jc[u] = (k < L) ? __builtin_nontemporal_load(&I->col[base + (int64_t)k * 64]) : 0;
  }
#pragma unroll
  for (int u = 0; u < kHdPer; ++u) {
    const int k = s0 + 8 * u;
    const bool ok = k < L;
    a[u] = ok ? __builtin_nontemporal_load(&I->A[base + (int64_t)k * 64]) : 0.0;
    b[u] = ok ? __builtin_nontemporal_load(&I->B[base + (int64_t)k * 64]) : 0.0;
    sg[u] = ok ? s[jc[u]] : 0;
  }
#pragma unroll
  for (int u = 0; u < kHdPer; ++u) {
    const int k = kHdChunk + s0 + 8 * u;
    jc[u] = (k < L) ? __builtin_nontemporal_load(&I->col[base + (int64_t)k * 64]) : 0;
  }
  for (int32_t k0 = 0; k0 < Lw; k0 += kHdChunk) {
#pragma unroll
    for (int u = 0; u < kHdPer; ++u) {
      const int e = (s0 + 8 * u) * R + r;
      sa[e] = (sg[u] > 0) ? a[u] : -a[u];
      sb[e] = (sg[u] > 0) ? b[u] : -b[u];
    }
    __syncthreads();
    // the next chunk's couplings and spins, and the columns after it, are
    // loaded while the current chunk is added
    const int32_t k1 = k0 + kHdChunk;
#pragma unroll
    for (int u = 0; u < kHdPer; ++u) {
      const int k = k1 + s0 + 8 * u;
      const bool ok = k < L;
      a[u] = ok ? __builtin_nontemporal_load(&I->A[base + (int64_t)k * 64]) : 0.0;
      b[u] = ok ? __builtin_nontemporal_load(&I->B[base + (int64_t)k * 64]) : 0.0;
      sg[u] = ok ? s[jc[u]] : 0;
    }
#pragma unroll
    for (int u = 0; u < kHdPer; ++u) {
      const int k = k1 + kHdChunk + s0 + 8 * u;
      jc[u] = (k < L) ? __builtin_nontemporal_load(&I->col[base + (int64_t)k * 64]) : 0;
    }
    if (tid < R && k0 < L) {
      // the chunk's sum from zero, then added to the row's (canonical order)
      const int kn = L - k0 < kHdChunk ? L - k0 : kHdChunk;
      double cp = 0.0, cq = 0.0;
      for (int kk = 0; kk < kn; ++kk) {
        cp += sa[kk * R + tid];
        cq += sb[kk * R + tid];
      }
      p += cp;
      pq += cq;
    }
    __syncthreads();
  }
  if (tid >= 64) return;
  uint32_t payload = 0;
  double key = 0.0;
  if (tid < R && i < I->n) key = field_finish(I, i, Rn->t, p, pq, payload);
  if (S == 1) {
    double mk = key;
    uint32_t mp = payload;
    wave_argmax(mk, mp);
    if (tid == 0) {
      I->t1key[row0 >> 6] = mk;
      I->t1idx[row0 >> 6] = mp;
    }
  }
  const unsigned long long bal = __ballot(key > 0.0);
  if (bal) {
    int pbase = 0;
    if (tid == 0) pbase = atomicAdd(I->ccount, __popcll(bal));
    pbase = __builtin_amdgcn_readfirstlane(pbase);
    pool_put(I, key, payload, bal, pbase);
  }
}

// The high-degree pass split over the 64-slot chunks, for instances too
// small to fill the device with k_field_hd (each of whose workgroups walks
// its rows' chunks one round trip after another).  k_field_hd_part: a
// 512-thread workgroup per (64-row slice, chunk) loads the chunk's slots of
// its rows (eight per thread, couplings and columns together, then the
// spins), stages the signed couplings in LDS, and the lane of each row adds
// its chunk in ascending slot order from zero; the sums go to I->part.
// k_field_hd_comb: a lane per row adds its chunk sums in ascending order --
// the canonical order of every pass -- then finishes the row (Eq. 2, the
// key), and each wavefront writes its 64 rows' maximum for the relax tree.
__global__ __launch_bounds__(512) void k_field_hd_part(const InstDev* __restrict__ insts,
                                                       RunDev* __restrict__ runs) {
  __shared__ double sa[kHdChunk * 64];
  __shared__ double sb[kHdChunk * 64];
  if (!runs->active) return;
  const InstDev* I = insts;
  const int nch = I->nch;
  const int64_t slice = blockIdx.x / nch;
  const int g = (int)(blockIdx.x % nch);
  const int64_t row0 = slice * 64;
  if (row0 >= I->n) return;
  const int tid = threadIdx.x;
  const int r = tid & 63;   // the thread's row in the slice
  const int s0 = tid >> 6;  // its first slot in the chunk; then every 8th
  const int64_t i = row0 + r;
  const int32_t L = (i < I->n) ? I->len[i] : 0;
  const int64_t base = slot_of(row0, I->D, 0) + r;  // slot 0 of the thread's row
  const int k0 = g * kHdChunk;
  const int8_t* __restrict__ s = I->s;
  int32_t jc[kHdPer];
  double a[kHdPer], b[kHdPer];
  int sg[kHdPer];
#pragma unroll
  for (int u = 0; u < kHdPer; ++u) {
    const int k = k0 + s0 + 8 * u;
    const bool ok = k < L;
    jc[u] = ok ? __builtin_nontemporal_load(&I->col[base + (int64_t)k * 64]) : 0;
    a[u] = ok ? __builtin_nontemporal_load(&I->A[base + (int64_t)k * 64]) : 0.0;
    b[u] = ok ? __builtin_nontemporal_load(&I->B[base + (int64_t)k * 64]) : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kHdPer; ++u) sg[u] = (k0 + s0 + 8 * u < L) ? s[jc[u]] : 0;
#pragma unroll
  for (int u = 0; u < kHdPer; ++u) {
    const int e = (s0 + 8 * u) * 64 + r;
    sa[e] = (sg[u] > 0) ? a[u] : -a[u];
    sb[e] = (sg[u] > 0) ? b[u] : -b[u];
  }
  __syncthreads();
  if (tid < 64 && k0 < L) {
    const int kn = L - k0 < kHdChunk ? L - k0 : kHdChunk;
    double cp = 0.0, cq = 0.0;
    for (int kk = 0; kk < kn; ++kk) {
      cp += sa[kk * 64 + tid];
      cq += sb[kk * 64 + tid];
    }
    I->part[(int64_t)g * I->n + i] = make_double2(cp, cq);
  }
}

__global__ __launch_bounds__(256) void k_field_hd_comb(const InstDev* __restrict__ insts,
                                                       RunDev* __restrict__ runs) {
  const RunDev* Rn = runs;
  if (!Rn->active) return;
  const InstDev* I = insts;
  const int lane = threadIdx.x & 63;
  const int64_t g64 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t row0 = g64 << 6;
  if (row0 >= I->n) return;
  const int64_t i = row0 + lane;
  uint32_t payload = 0;
  double key = 0.0;
  if (i < I->n) {
    const int32_t L = I->len[i];
    double p = 0.0, pq = 0.0;
    for (int c = 0; c * kHdChunk < L; ++c) {
      const double2 v = I->part[(int64_t)c * I->n + i];
      p += v.x;
      pq += v.y;
    }
    key = field_finish(I, i, Rn->t, p, pq, payload);
  }
  double mk = key;
  uint32_t mp = payload;
  wave_argmax(mk, mp);
  if (lane == 0) {
    I->t1key[g64] = mk;
    I->t1idx[g64] = mp;
  }
  const unsigned long long bal = __ballot(key > 0.0);
  if (bal) {
    int pbase = 0;
    if (lane == 0) pbase = atomicAdd(I->ccount, __popcll(bal));
    pbase = __builtin_amdgcn_readfirstlane(pbase);
    pool_put(I, key, payload, bal, pbase);
  }
}

// Per-64-row maxima of the keys a split high-degree pass wrote (one
// wavefront per 64 rows), for the relax tree.
__global__ __launch_bounds__(256) void k_slice_max(const InstDev* __restrict__ insts,
                                                   RunDev* __restrict__ runs) {
  if (!runs->active) return;
  const InstDev* I = insts;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t i = (g << 6) + lane;
  if ((g << 6) >= I->n) return;
  double k = 0.0;
  uint32_t pay = 0u;
  if (i < I->n) {
    k = I->key[i];
    pay = (uint32_t)i | (I->s[i] < 0 ? 0x80000000u : 0u);
  }
  wave_argmax(k, pay);
  if (lane == 0) {
    I->t1key[g] = k;
    I->t1idx[g] = pay;
  }
}

// ------------------------------------------------------------ relax
struct RelaxLds {
  double* l1k;                // first level: maximum key of each tile
  uint32_t* l1i;              //   its index | sign bit
  int32_t* l1flag;            //   tile touched by the current flip
  unsigned long long* l1nk;   //   largest new key of the flip's updates (bits), 0: none
  unsigned long long* l1ni;   //   lowest (index << 1 | spin<0) among updates with that key
  int32_t* l1resc;            //   the tile's maximum was updated: rescan it
  int32_t* l1rlist;           //   tiles to rescan
  double* l2k;                // second level: maximum over 64 tiles
  uint32_t* l2i;
  int32_t* l2flag;            //   group touched by the current flip
};

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

__host__ __device__ inline size_t relax_tree_lds_bytes(int64_t n, int32_t l1_shift) {
  const int64_t nt1 = (n + (1LL << l1_shift) - 1) >> l1_shift;
  const int64_t nt2 = (nt1 + kL2Group - 1) / kL2Group;
  size_t off = 0;
  off = align16(off + sizeof(unsigned long long) * nt1);
  off = align16(off + sizeof(unsigned long long) * nt1);
  off = align16(off + sizeof(double) * nt1);
  off = align16(off + sizeof(uint32_t) * nt1);
  for (int a = 0; a < 3; ++a) off = align16(off + sizeof(int32_t) * nt1);
  off = align16(off + sizeof(double) * nt2);
  off = align16(off + sizeof(uint32_t) * nt2);
  off = align16(off + sizeof(int32_t) * nt2);
  return off;
}

__device__ inline RelaxLds carve(unsigned char* base, int nt1, int nt2) {
  RelaxLds L;
  size_t off = 0;
  L.l1nk = (unsigned long long*)(base + off);
  off = align16(off + sizeof(unsigned long long) * nt1);
  L.l1ni = (unsigned long long*)(base + off);
  off = align16(off + sizeof(unsigned long long) * nt1);
  L.l1k = (double*)(base + off);
  off = align16(off + sizeof(double) * nt1);
  L.l1i = (uint32_t*)(base + off);
  off = align16(off + sizeof(uint32_t) * nt1);
  L.l1flag = (int32_t*)(base + off);
  off = align16(off + sizeof(int32_t) * nt1);
  L.l1resc = (int32_t*)(base + off);
  off = align16(off + sizeof(int32_t) * nt1);
  L.l1rlist = (int32_t*)(base + off);
  off = align16(off + sizeof(int32_t) * nt1);
  L.l2k = (double*)(base + off);
  off = align16(off + sizeof(double) * nt2);
  L.l2i = (uint32_t*)(base + off);
  off = align16(off + sizeof(uint32_t) * nt2);
  L.l2flag = (int32_t*)(base + off);
  return L;
}

struct RelaxShared {
  int nr;  // tiles to rescan
  int pause;  // the relax stops here and resumes in a later launch
  double key;
  uint32_t pay;
  // predicted next flip: high 32 bits of the best updated key, then its index
  unsigned long long pfk;
  // runner-up of the tree before the flip (j's own tile left out), packed the
  // same way; 0 when none is known
  unsigned long long ruk;
};

// True once the deadline (device constant-rate clock; 0: none) has passed.
__device__ inline bool past(uint64_t deadline) {
  return deadline != 0 && (uint64_t)wall_clock64() > deadline;
}

// ------------------------------------------------------------ speculative relax
// Exact-order batched relax for steps that start with many flippable
// magnets.  Candidates live in a pool in memory (filled by the field phase)
// and a hot window in LDS that is sorted best first (largest key, then lowest
// index).  Entries are (key, index | sign bit, version); an entry is valid
// while its version equals the magnet's version counter, which every change
// of the magnet's key bumps.  Every valid pool entry is no better than
// cold_max, so window entries better than cold_max can be taken in order.
//
// A batch takes the first B safe window entries c_1 .. c_B and flips the
// longest prefix c_1 .. c_p that the one-at-a-time relax would flip in the
// same order: the members and their neighbour sets are pairwise disjoint
// (so no member's field or key depends on an earlier member of the prefix,
// and every touched magnet gets exactly one update), and no touched magnet's
// new key beats a later member of the prefix.  Then c_m is the argmax after
// c_1 .. c_{m-1} for every m <= p, and applying the prefix together gives
// the same flips, log, fields and keys, bit for bit.
constexpr int kWin = 2048;        // hot window entries
constexpr int kHash = 4096;       // conflict table slots
constexpr int kMaxPairs = 2048;   // member + neighbour slots per batch
constexpr int kMaxMembers = 64;
// A step whose first kSwitchBatches batches commit fewer than spec_switch
// (2.5 unless overridden) flips each on average -- an avalanche: every flip
// makes a neighbour the next candidate -- continues on the max tree, which
// costs about half a batch per flip on such steps.
constexpr int kSwitchBatches = 16;

// Relax order of two magnets: larger key first, then lower index.
__device__ inline bool better(double ka, uint32_t pa, double kb, uint32_t pb) {
  return ka > kb || (ka == kb && (pa & 0x7fffffffu) < (pb & 0x7fffffffu));
}

// Order of pool and window entries: the relax order, then the newer version
// of the same magnet first, so that no two distinct entries tie.
__device__ inline bool better_e(double ka, uint32_t pa, uint32_t va, double kb, uint32_t pb,
                                uint32_t vb) {
  if (ka != kb) return ka > kb;
  const uint32_t ia = pa & 0x7fffffffu, ib = pb & 0x7fffffffu;
  if (ia != ib) return ia < ib;
  return va > vb;
}

struct SpecLds {
  unsigned char* win;  // hot window, two buffers of kWin entries each:
                       //   buffer b: keys at win + b * kWinBytes, then payloads, versions
  double* sk;       // staging / sort scratch (aliases the conflict table)
  uint32_t* sp;
  uint32_t* sv;
  uint32_t* hidx;   // conflict table: magnet + 1 (0: empty)
  int32_t* hown;    //   lowest member rank owning that magnet
  int32_t* mval;    // per window position: member valid
  int32_t* mrank;   //   its rank among the valid members (-1: stale)
  double* mk;       // per rank: key, payload, window position
  uint32_t* mp;
  int32_t* mpos;
};

constexpr size_t kWinBytes = (size_t)kWin * 16;
__device__ inline double* win_k(const SpecLds& S, int b) {
  return (double*)(S.win + (size_t)b * kWinBytes);
}
__device__ inline uint32_t* win_p(const SpecLds& S, int b) {
  return (uint32_t*)(S.win + (size_t)b * kWinBytes + sizeof(double) * kWin);
}
__device__ inline uint32_t* win_v(const SpecLds& S, int b) {
  return (uint32_t*)(S.win + (size_t)b * kWinBytes + (sizeof(double) + sizeof(uint32_t)) * kWin);
}

__host__ __device__ inline size_t spec_lds_bytes() {
  return 2 * (size_t)kWin * 16 + (size_t)kWin * 16 + (size_t)kMaxMembers * (4 + 4 + 8 + 4 + 4);
}

__device__ inline SpecLds carve_spec(unsigned char* base) {
  SpecLds S;
  S.win = base;
  size_t off = 2 * kWinBytes;
  S.sk = (double*)(base + off);
  S.sp = (uint32_t*)(base + off + sizeof(double) * kWin);
  S.sv = (uint32_t*)(base + off + (sizeof(double) + sizeof(uint32_t)) * kWin);
  S.hidx = (uint32_t*)(base + off);
  S.hown = (int32_t*)(base + off + sizeof(uint32_t) * kHash);
  off += (size_t)kWin * 16;
  S.mk = (double*)(base + off);
  off += sizeof(double) * kMaxMembers;
  S.mp = (uint32_t*)(base + off);
  off += sizeof(uint32_t) * kMaxMembers;
  S.mpos = (int32_t*)(base + off);
  off += sizeof(int32_t) * kMaxMembers;
  S.mval = (int32_t*)(base + off);
  off += sizeof(int32_t) * kMaxMembers;
  S.mrank = (int32_t*)(base + off);
  return S;
}

struct SpecShared {
  int nx, xb, ns, nvalid, p, safe, cb, pause, npow;
  int64_t ncold, ncold_out, napp;
  double cmk;       // cold_max (key, payload, version); key -1: pool empty
  uint32_t cmp, cmv;
  double rk;        // best entry a merge discarded into the pool
  uint32_t rp, rv;
  double tau;       // refill threshold (selective refill)
  int over;         // selective refill: more entries above tau than fit
  double wk[16];    // per-wavefront best entries (selective refill)
  uint32_t wp[16], wv[16];
};

// Block-wide bitonic sort, best first, of P (a power of two) entries.
__device__ __forceinline__ void bitonic_best_first(double* k, uint32_t* p, uint32_t* v, int P) {
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int q = tid; q < P / 2; q += NT) {
        const int lo = 2 * stride * (q / stride) + (q % stride);
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;  // this segment runs best first
        const bool sw = up ? better_e(k[hi], p[hi], v[hi], k[lo], p[lo], v[lo])
                           : better_e(k[lo], p[lo], v[lo], k[hi], p[hi], v[hi]);
        if (sw) {
          const double tk = k[lo];
          k[lo] = k[hi];
          k[hi] = tk;
          const uint32_t tp = p[lo];
          p[lo] = p[hi];
          p[hi] = tp;
          const uint32_t tv = v[lo];
          v[lo] = v[hi];
          v[hi] = tv;
        }
      }
      __syncthreads();
    }
  }
}

// Number of entries taken from A among the first d outputs of merge(A, B)
// (both best first; on equal entries A goes first).
__device__ __forceinline__ int co_rank(int d, const double* ak, const uint32_t* ap,
                                      const uint32_t* av, int na, const double* bk,
                                      const uint32_t* bp, const uint32_t* bv, int nb) {
  int lo = d > nb ? d - nb : 0;
  int hi = d < na ? d : na;
  while (lo < hi) {
    const int i = (lo + hi) >> 1;
    const int j = d - i;
    if (j > 0 && i < na && !better_e(bk[j - 1], bp[j - 1], bv[j - 1], ak[i], ap[i], av[i]))
      lo = i + 1;
    else
      hi = i;
  }
  return lo;
}

// Merge A = window[a0, a0+na) with B = staging[0, nb) (both best first):
// the first `keep` outputs become the window (other buffer), the rest are
// appended to pool buffer pb at sh.ncold_out; sh.rk/rp keeps the best entry
// sent to the pool.
__device__ __forceinline__ void merge_keep(const InstDev* I, const SpecLds& S, SpecShared& sh, int a0, int na,
                           int nb, int keep, int pb) {
  const int tid = threadIdx.x, NT = blockDim.x;
  const int xb = sh.xb;
  const double* ak = win_k(S, xb) + a0;
  const uint32_t* ap = win_p(S, xb) + a0;
  const uint32_t* av = win_v(S, xb) + a0;
  double* ok = win_k(S, xb ^ 1);
  uint32_t* op = win_p(S, xb ^ 1);
  uint32_t* ov = win_v(S, xb ^ 1);
  uint32_t* pool_p = I->cpay[pb];
  double* pool_k = I->ckey[pb];
  uint32_t* pool_v = I->cver[pb];
  const int total = na + nb;
  const int per = (total + NT - 1) / NT;
  const int d0 = tid * per < total ? tid * per : total;
  const int d1 = d0 + per < total ? d0 + per : total;
  const int64_t base = sh.ncold_out;
  if (d0 < d1) {
    int i = co_rank(d0, ak, ap, av, na, S.sk, S.sp, S.sv, nb);
    int j = d0 - i;
    for (int d = d0; d < d1; ++d) {
      double ek;
      uint32_t epay, ever;
      if (j >= nb || (i < na && !better_e(S.sk[j], S.sp[j], S.sv[j], ak[i], ap[i], av[i]))) {
        ek = ak[i];
        epay = ap[i];
        ever = av[i];
        ++i;
      } else {
        ek = S.sk[j];
        epay = S.sp[j];
        ever = S.sv[j];
        ++j;
      }
      if (d < keep) {
        ok[d] = ek;
        op[d] = epay;
        ov[d] = ever;
      } else {
        const int64_t q = base + (d - keep);
        pool_k[q] = ek;
        pool_p[q] = epay;
        pool_v[q] = ever;
        if (d == keep && better_e(ek, epay, ever, sh.rk, sh.rp, sh.rv)) {
          sh.rk = ek;
          sh.rp = epay;
          sh.rv = ever;
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    sh.ncold_out += total - keep;
    sh.xb ^= 1;
    sh.nx = keep;
  }
  __syncthreads();
}

// Sort staging entries [0, ns) best first.  Up to one entry per thread:
// each thread counts the entries that beat its own (every thread reads the
// same entry at a time, a broadcast) and moves it to that rank; no two
// entries tie under the pool order.  Larger sets: bitonic sort, padded to a
// power of two.
__device__ __forceinline__ void sort_staging(const SpecLds& S, int ns) {
  const int tid = threadIdx.x;
  if (ns <= (int)blockDim.x) {
    double k = 0.0;
    uint32_t p = 0, v = 0;
    int rank = 0;
    if (tid < ns) {
      k = S.sk[tid];
      p = S.sp[tid];
      v = S.sv[tid];
      for (int q = 0; q < ns; ++q) rank += better_e(S.sk[q], S.sp[q], S.sv[q], k, p, v) ? 1 : 0;
    }
    __syncthreads();
    if (tid < ns) {
      S.sk[rank] = k;
      S.sp[rank] = p;
      S.sv[rank] = v;
    }
    __syncthreads();
    return;
  }
  int P = 1;
  while (P < ns) P <<= 1;
  for (int q = ns + tid; q < P; q += blockDim.x) {
    S.sk[q] = -1.0;
    S.sp[q] = 0x7fffffffu;
    S.sv[q] = 0u;
  }
  __syncthreads();
  bitonic_best_first(S.sk, S.sp, S.sv, P);
}

// Window := best kWin entries of (window + valid pool entries); the other
// valid pool entries move to the other pool buffer; cold_max becomes exact.
__device__ __forceinline__ void refill(const InstDev* I, const SpecLds& S, SpecShared& sh) {
  const int tid = threadIdx.x, NT = blockDim.x;
  const int cb = sh.cb;
  const int64_t ncold = sh.ncold;
  if (tid == 0) {
    sh.ncold_out = 0;
    sh.rk = -1.0;
    sh.rp = 0x7fffffffu;
    sh.rv = 0u;
  }
  __syncthreads();
  for (int64_t c0 = 0; c0 < ncold; c0 += kWin) {
    const int m = (int)(ncold - c0 < kWin ? ncold - c0 : kWin);
    for (int q = tid; q < m; q += NT) {
      const uint32_t pay = I->cpay[cb][c0 + q];
      const uint32_t ver = I->cver[cb][c0 + q];
      const bool ok = I->ver[pay & 0x7fffffffu] == ver;
      S.sk[q] = ok ? I->ckey[cb][c0 + q] : -1.0;
      S.sp[q] = ok ? pay : 0x7fffffffu;
      S.sv[q] = ok ? ver : (uint32_t)q;  // invalid entries: distinct, sorted last
    }
    __syncthreads();
    sort_staging(S, m);
    if (tid == 0) {
      int lo = 0, hi = m;  // valid entries sort first
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (S.sk[mid] > 0.0) lo = mid + 1; else hi = mid;
      }
      sh.ns = lo;
    }
    __syncthreads();
    const int nv = sh.ns;
    const int nx = sh.nx;
    const int keep = nx + nv < kWin ? nx + nv : kWin;
    merge_keep(I, S, sh, 0, nx, nv, keep, cb ^ 1);
  }
  if (tid == 0) {
    sh.cb = cb ^ 1;
    sh.ncold = sh.ncold_out;
    sh.cmk = sh.rk;
    sh.cmp = sh.rp;
    sh.cmv = sh.rv;
  }
  __syncthreads();
}

// Refill for a large pool: a threshold tau from a sorted sample of the
// pool's keys puts about kWin / 2 entries above it; one pass drops stale
// entries, sends the current ones above tau to staging and those at or
// below tau to the other pool buffer, keeping the best of those (pool
// order) as the cold bound; staging is sorted and merged into the window,
// whose overflow joins the pool and the bound, which stays exact.  Only
// about kWin entries are sorted instead of the whole pool.  If more current
// entries than staging holds lie above tau, or none does, the pass is
// discarded and the full refill runs instead.
__device__ __forceinline__ void refill_select(const InstDev* I, const SpecLds& S, SpecShared& sh) {
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int cb = sh.cb;
  const int64_t ncold = sh.ncold;
  for (int q = tid; q < kWin; q += NT) {
    S.sk[q] = I->ckey[cb][(int64_t)q * ncold / kWin];
    S.sp[q] = (uint32_t)q;
    S.sv[q] = 0u;
  }
  __syncthreads();
  bitonic_best_first(S.sk, S.sp, S.sv, kWin);
  if (tid == 0) {
    int r = (int)((int64_t)(kWin / 2) * kWin / ncold);
    if (r < 1) r = 1;
    sh.tau = S.sk[r];
    sh.ns = 0;
    sh.over = 0;
    sh.ncold_out = 0;
    sh.rk = -1.0;
    sh.rp = 0x7fffffffu;
    sh.rv = 0u;
  }
  __syncthreads();
  const double tau = sh.tau;
  const unsigned long long lt = (1ull << lane) - 1ull;
  double bk = -1.0;
  uint32_t bp = 0x7fffffffu, bv = 0u;
  for (int64_t q0 = 0; q0 < ncold; q0 += NT) {
    const int64_t q = q0 + tid;
    bool up = false, down = false;
    double k = 0.0;
    uint32_t pay = 0, ver = 0;
    if (q < ncold) {
      k = I->ckey[cb][q];
      pay = I->cpay[cb][q];
      ver = I->cver[cb][q];
      const bool cur = I->ver[pay & 0x7fffffffu] == ver;
      up = cur && k > tau;
      down = cur && !(k > tau);
    }
    const unsigned long long bu = __ballot(up), bd = __ballot(down);
    int ubase = 0, dbase = 0;
    if (lane == 0) {
      if (bu) ubase = atomicAdd(&sh.ns, __popcll(bu));
      if (bd) dbase = (int)atomicAdd((unsigned long long*)&sh.ncold_out, (unsigned long long)__popcll(bd));
    }
    ubase = __builtin_amdgcn_readfirstlane(ubase);
    dbase = __builtin_amdgcn_readfirstlane(dbase);
    if (up) {
      const int pos = ubase + __popcll(bu & lt);
      if (pos < kWin) {
        S.sk[pos] = k;
        S.sp[pos] = pay;
        S.sv[pos] = ver;
      } else {
        sh.over = 1;
      }
    }
    if (down) {
      const int64_t pos = dbase + __popcll(bd & lt);
      I->ckey[cb ^ 1][pos] = k;
      I->cpay[cb ^ 1][pos] = pay;
      I->cver[cb ^ 1][pos] = ver;
      if (better_e(k, pay, ver, bk, bp, bv)) {
        bk = k;
        bp = pay;
        bv = ver;
      }
    }
  }
  // best entry sent down: per wavefront, then over the wavefronts
  for (int off = 32; off > 0; off >>= 1) {
    const double ok = __shfl_down(bk, off);
    const uint32_t op = __shfl_down(bp, off), ov = __shfl_down(bv, off);
    if (lane + off < 64 && better_e(ok, op, ov, bk, bp, bv)) {
      bk = ok;
      bp = op;
      bv = ov;
    }
  }
  if (lane == 0) {
    sh.wk[wave] = bk;
    sh.wp[wave] = bp;
    sh.wv[wave] = bv;
  }
  __syncthreads();
  // Too many current entries above tau, or none (ties at the top of the
  // sample can put tau on the best key): the full refill, from the same pool.
  if (sh.over || sh.ns == 0) {
    refill(I, S, sh);
    return;
  }
  if (tid == 0) {
    for (int w = 0; w < (NT >> 6); ++w)
      if (better_e(sh.wk[w], sh.wp[w], sh.wv[w], sh.rk, sh.rp, sh.rv)) {
        sh.rk = sh.wk[w];
        sh.rp = sh.wp[w];
        sh.rv = sh.wv[w];
      }
  }
  __syncthreads();
  const int ns = sh.ns;
  sort_staging(S, ns);
  const int nx = sh.nx;
  const int keep = nx + ns < kWin ? nx + ns : kWin;
  merge_keep(I, S, sh, 0, nx, ns, keep, cb ^ 1);
  if (tid == 0) {
    sh.cb = cb ^ 1;
    sh.ncold = sh.ncold_out;
    sh.cmk = sh.rk;
    sh.cmp = sh.rp;
    sh.cmv = sh.rv;
  }
  __syncthreads();
}


// Window entries better than cold_max (all of them when the pool is
// empty), counted by one wavefront (every lane gets the count): the safe
// entries are a prefix of the window, so 64 segment ends locate the
// boundary's segment, and one lane per entry of that segment finds it.
__device__ __forceinline__ int count_safe_wave(const SpecLds& S, const SpecShared& sh) {
  const int lane = threadIdx.x & 63;
  const int nx = sh.nx;
  if (sh.ncold == 0 || nx == 0) return nx;
  const double* k = win_k(S, sh.xb);
  const uint32_t* p = win_p(S, sh.xb);
  const uint32_t* v = win_v(S, sh.xb);
  const double cmk = sh.cmk;
  const uint32_t cmp = sh.cmp, cmv = sh.cmv;
  const int step = (nx + 63) >> 6;
  const int e = (lane + 1) * step - 1;
  const bool ok = e < nx && better_e(k[e], p[e], v[e], cmk, cmp, cmv);
  const int c = __popcll(__ballot(ok));
  const int e2 = c * step + lane;
  const bool ok2 = lane < step && e2 < nx && better_e(k[e2], p[e2], v[e2], cmk, cmp, cmv);
  return c * step + __popcll(__ballot(ok2));
}

__device__ inline uint32_t hash_slot(uint32_t i) { return (i * 2654435761u) >> (32 - 12); }

// Relax at step t in speculative batches (needs 1024 threads).  flips,
// logpos and hash are the running counters (hash significant in thread 0).
// Returns 0, -5 (flip cap reached with a flippable magnet left),
// 1 (deadline passed after at least one batch, flippable magnets left) or
// 2 (after kSwitchBatches batches the mean batch is below spec_switch flips:
// the flippable magnets crowd each other's neighbourhoods, and the step
// goes on one flip at a time).
__device__ __forceinline__ int relax_spec(const InstDev* __restrict__ I, int64_t t, unsigned char* lds,
                          SpecShared& sh, int64_t ncand, int64_t& flips, int64_t& logpos,
                          uint64_t& hash, uint64_t deadline) {
  constexpr int kPPT = kMaxPairs / 1024;  // pair slots per thread
  const int tid = threadIdx.x, NT = blockDim.x;
  SpecLds S = carve_spec(lds);
  const int32_t D = I->D;
  const int32_t mode = I->field_mode;
  const double pb = I->b, pc = I->c, ep = I->e_par, eq = I->e_perp;
  const int64_t max_flips = I->max_flips;
  const int PW = D + 1;  // pair slots per member: its neighbours and itself
  int Bmax = kMaxPairs / PW;
  if (Bmax > kMaxMembers) Bmax = kMaxMembers;
  // Members taken per batch: about twice the last committed prefix, since
  // the members past the prefix only cost loads and key evaluations;
  // doubled while whole batches commit.
  int bcap = Bmax;
  if (tid == 0) {
    sh.nx = 0;
    sh.xb = 0;
    sh.cb = 0;
    sh.ncold = ncand;
    sh.cmk = 1e300;  // unknown until the first refill
    sh.cmp = 0;
    sh.cmv = 0;
  }
  __syncthreads();
  int status = 0;
  const int64_t flips0 = flips;
  int nbatch = 0;
  while (true) {
    if (nbatch >= kSwitchBatches && (double)(flips - flips0) < I->spec_switch * nbatch) {
      status = 2;
      break;
    }
    if (tid < 64) {
      const int sf = count_safe_wave(S, sh);
      if (tid == 0) {
        sh.safe = sf;
        sh.pause = (flips > flips0 && past(deadline)) ? 1 : 0;
      }
    }
    __syncthreads();
    const int pause = sh.pause;
    if (sh.safe == 0 || sh.ncold + kMaxPairs + kWin > I->ccap) {
      if (sh.ncold == 0 && sh.safe == 0) break;
      if (sh.ncold > 4 * kWin)
        refill_select(I, S, sh);
      else
        refill(I, S, sh);
      if (tid < 64) {
        const int sf = count_safe_wave(S, sh);
        if (tid == 0) sh.safe = sf;
      }
      __syncthreads();
      if (sh.safe == 0) break;  // the pool held stale entries only
    }
    if (pause) {  // flippable magnets remain
      status = 1;
      break;
    }
    const int B = sh.safe < bcap ? sh.safe : bcap;
    const int xb = sh.xb;
    const double* xk = win_k(S, xb);
    const uint32_t* xp = win_p(S, xb);
    const uint32_t* xv = win_v(S, xb);
    // ---- round trip 1: member versions and the members' neighbour slots
    int pr_m[kPPT], pr_i[kPPT];
    double pr_a[kPPT], pr_b[kPPT];
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {
      pr_m[u] = -1;
      pr_i[u] = -1;
      pr_a[u] = 0.0;
      pr_b[u] = 0.0;
      const int q = tid + u * NT;
      if (q < B * PW) {
        const int m = q / PW, k = q % PW;
        const uint32_t j = xp[m] & 0x7fffffffu;
        pr_m[u] = m;
        if (k == D) {
          pr_i[u] = (int)j;
        } else {
          const int64_t sl = (int64_t)j * D + k;
          pr_i[u] = I->rcol[sl];
          pr_a[u] = I->rA[sl];
          pr_b[u] = I->rBr[sl];
        }
      }
    }
    if (tid < B) S.mval[tid] = (I->ver[xp[tid] & 0x7fffffffu] == xv[tid]) ? 1 : 0;
    for (int q = tid; q < kHash; q += NT) {
      S.hidx[q] = 0u;
      S.hown[q] = 0x7fffffff;
    }
    __syncthreads();
    if (tid < 64) {  // ranks of the valid members, one wavefront
      const bool v = tid < B && S.mval[tid] != 0;
      const unsigned long long bal = __ballot(v);
      const int r = __popcll(bal & ((1ull << tid) - 1ull));
      if (tid < B) S.mrank[tid] = v ? r : -1;
      if (v) {
        S.mk[r] = xk[tid];
        S.mp[r] = xp[tid];
        S.mpos[r] = tid;
      }
      if (tid == 0) {
        sh.nvalid = __popcll(bal);
        sh.p = __popcll(bal);
        sh.ns = 0;
        sh.napp = 0;
        sh.npow = 0;
      }
    }
    __syncthreads();
    const int nvalid = sh.nvalid;
    int pr_r[kPPT];
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {
      pr_r[u] = (pr_m[u] >= 0) ? S.mrank[pr_m[u]] : -1;
      if (pr_i[u] < 0) pr_r[u] = -1;  // padding slot
    }
    // ---- pairwise disjoint neighbour sets: lowest owning rank per magnet
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {
      if (pr_r[u] >= 0) {
        const uint32_t want = (uint32_t)pr_i[u] + 1u;
        uint32_t s = hash_slot((uint32_t)pr_i[u]);
        while (true) {
          const uint32_t old = atomicCAS(&S.hidx[s], 0u, want);
          if (old == 0u || old == want) break;
          s = (s + 1) & (kHash - 1);
        }
        atomicMin(&S.hown[s], pr_r[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {
      if (pr_r[u] >= 0) {
        const uint32_t want = (uint32_t)pr_i[u] + 1u;
        uint32_t s = hash_slot((uint32_t)pr_i[u]);
        while (S.hidx[s] != want) s = (s + 1) & (kHash - 1);
        if (S.hown[s] < pr_r[u]) atomicMin(&sh.p, pr_r[u]);
      }
    }
    __syncthreads();
    const int p_ab = sh.p;
    // ---- round trip 2: touched magnets of the conflict-free prefix.  Keys
    // the switching bound cannot settle go through a dense list in LDS
    // (aliasing the conflict table, done with), so that the FP64 powers run
    // on full wavefronts.
    double nh_p[kPPT], nh_q[kPPT], nkey[kPPT], nd_p[kPPT], nd_q[kPPT];
    uint32_t nver[kPPT];
    int nsi[kPPT], ppos[kPPT];
    double* pw_a = S.sk;            // kMaxPairs doubles
    double* pw_q = (double*)S.sp;   // kMaxPairs doubles (sp and sv)
    double pa[kPPT], pq[kPPT];
    bool need[kPPT];
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {  // all gathers first: one round trip
      nkey[u] = 0.0;
      ppos[u] = -1;
      pa[u] = 0.0;
      pq[u] = 0.0;
      need[u] = false;
      const int k = (pr_m[u] >= 0) ? (tid + u * NT) % PW : D;
      if (pr_r[u] >= 0 && pr_r[u] < p_ab && k < D) {
        const int i = pr_i[u];
        const uint32_t mpay = S.mp[pr_r[u]];
        const double two = (mpay & 0x80000000u) ? 2.0 : -2.0;  // s_new = -s_old
        const double da = two * pr_a[u], db = two * pr_b[u];
        const double2 hi = I->h[i];
        nh_p[u] = hi.x + da;
        nh_q[u] = hi.y + db;
        if (mode == kFieldCarry) {
          const double2 di = I->hd[i];
          nd_p[u] = di.x + da;
          nd_q[u] = di.y + db;
        }
        nsi[u] = I->s[i];
        nver[u] = I->ver[i];
        need[u] = key_needs_powers(nsi[u], nh_p[u], nh_q[u], I->hk[i], pb, pc, ep, eq, pa[u],
                                   pq[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {
      const unsigned long long bal = __ballot(need[u]);
      if (bal) {
        int base = 0;
        if ((tid & 63) == 0) base = atomicAdd(&sh.npow, __popcll(bal));
        base = __builtin_amdgcn_readfirstlane(base);
        if (need[u]) {
          ppos[u] = base + __popcll(bal & ((1ull << (tid & 63)) - 1ull));
          pw_a[ppos[u]] = pa[u];
          pw_q[ppos[u]] = pq[u];
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < sh.npow; e += NT) pw_a[e] = key_from_powers(pw_a[e], pw_q[e], ep, eq);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {
      if (ppos[u] >= 0) {
        nkey[u] = pw_a[ppos[u]];
        const int i = pr_i[u];
        if (nkey[u] > 0.0) {
          // first later member of the prefix this magnet would beat
          const uint32_t npay = (uint32_t)i | (nsi[u] < 0 ? 0x80000000u : 0u);
          int lo = pr_r[u] + 1, hi = p_ab;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (better(nkey[u], npay, S.mk[mid], S.mp[mid])) hi = mid; else lo = mid + 1;
          }
          if (lo < p_ab) atomicMin(&sh.p, lo);
        }
      }
    }
    __syncthreads();
    int p = sh.p;
    if (p > max_flips - flips) p = (int)(max_flips - flips);
    if (p <= 0 && nvalid > 0) {
      status = -5;
      break;
    }
    // ---- commit members [0, p) and their neighbours
    if (tid < p) {
      const uint32_t mpay = S.mp[tid];
      const uint32_t j = mpay & 0x7fffffffu;
      I->s[j] = (mpay & 0x80000000u) ? (int8_t)1 : (int8_t)-1;
      I->key[j] = 0.0;
      I->ver[j] = xv[S.mpos[tid]] + 1u;
    }
    if (tid < 64) {  // log the members in order (one lane each), then fold them into the hash
      const uint32_t jr = (tid < p) ? (S.mp[tid] & 0x7fffffffu) : 0u;
      if (tid < p && logpos + tid < I->log_cap) {
        I->log_t[logpos + tid] = (int32_t)t;
        I->log_j[logpos + tid] = (int32_t)jr;
      }
      for (int r = 0; r < p; ++r) {
        const uint64_t w = ((uint64_t)(uint32_t)t << 32) |
                           (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)jr, r);
        hash = (hash ^ w) * 0x100000001b3ull;
      }
    }
    logpos += p;
    const double cmk = sh.cmk;
    const uint32_t cmp = sh.cmp, cmv = sh.cmv;
    const int cb = sh.cb;
    const int64_t ncold = sh.ncold;
    // flippable touched magnets go to staging (if they may enter the window)
    // or to the cold pool, with one LDS atomic per wavefront for each
    const unsigned long long lt = (1ull << (tid & 63)) - 1ull;
#pragma unroll
    for (int u = 0; u < kPPT; ++u) {
      const int k = (pr_m[u] >= 0) ? (tid + u * NT) % PW : D;
      bool st = false, co = false;
      uint32_t npay = 0, v1 = 0;
      if (pr_r[u] >= 0 && pr_r[u] < p && k < D) {
        const int i = pr_i[u];
        I->h[i] = make_double2(nh_p[u], nh_q[u]);
        if (mode == kFieldCarry) {
          I->hd[i] = make_double2(nd_p[u], nd_q[u]);
        } else if (mode == kFieldDirty) {
          I->dirty[i] = 1;
        }
        I->key[i] = nkey[u];
        v1 = nver[u] + 1u;
        I->ver[i] = v1;
        if (nkey[u] > 0.0) {
          npay = (uint32_t)i | (nsi[u] < 0 ? 0x80000000u : 0u);
          st = better_e(nkey[u], npay, v1, cmk, cmp, cmv);
          co = !st;
        }
      }
      const unsigned long long bs = __ballot(st), bc = __ballot(co);
      int sbase = 0, cbase = 0;
      if ((tid & 63) == 0) {
        if (bs) sbase = atomicAdd(&sh.ns, __popcll(bs));
        if (bc) cbase = (int)atomicAdd((unsigned long long*)&sh.napp, (unsigned long long)__popcll(bc));
      }
      sbase = __builtin_amdgcn_readfirstlane(sbase);
      cbase = __builtin_amdgcn_readfirstlane(cbase);
      if (st) {
        const int q = sbase + __popcll(bs & lt);
        S.sk[q] = nkey[u];
        S.sp[q] = npay;
        S.sv[q] = v1;
      }
      if (co) {
        const int64_t q = ncold + cbase + __popcll(bc & lt);
        I->ckey[cb][q] = nkey[u];
        I->cpay[cb][q] = npay;
        I->cver[cb][q] = v1;
      }
    }
    flips += p;
    ++nbatch;
    bcap = (p >= B) ? 2 * B : 2 * p + 2;
    if (bcap < 8) bcap = 8;
    if (bcap > Bmax) bcap = Bmax;
    __syncthreads();
    // window entries consumed: up to the last committed member (stale ones
    // in between included), or the whole batch when every valid member went
    const int consumed = (p < nvalid) ? S.mpos[p - 1] + 1 : B;
    const int ns = sh.ns;
    if (tid == 0) {
      sh.ncold += sh.napp;
      sh.ncold_out = sh.ncold;
      sh.rk = sh.cmk;
      sh.rp = sh.cmp;
      sh.rv = sh.cmv;
    }
    __syncthreads();
    sort_staging(S, ns);
    const int na = sh.nx - consumed;
    const int keep = na + ns < kWin ? na + ns : kWin;
    merge_keep(I, S, sh, consumed, na, ns, keep, sh.cb);
    if (tid == 0) {
      sh.ncold = sh.ncold_out;
      sh.cmk = sh.rk;
      sh.cmp = sh.rp;
      sh.cmv = sh.rv;
    }
    __syncthreads();
  }
  return status;
}

// Relax one instance at step t with the whole workgroup (Sec. II.H).  The
// flippable keys are kept in a three-level max tree: the key array in
// memory, first-level tiles of 2^l1_shift magnets and second-level groups of
// 64 tiles in LDS, built from the per-64-row maxima of the field phase
// (with kFlatOk, up to kFlatTiles tiles the root reads the tiles directly).
// Per flip: the root gives j; thread 0 flips it and logs it; the threads
// update j's neighbours (dipolar and total field += 2 s_new * coupling, new
// key); the touched tiles are brought up to date from the updates, or
// rescanned when their maximum fell, and then the touched groups.  Returns
// 0, -5 (flip cap reached with a flippable magnet left) or 1 (deadline
// passed, checked every 16 flips, with flippable magnets left).
template <bool kFlatOk>
__device__ __forceinline__ int relax_tree(const InstDev* __restrict__ I, int64_t t, unsigned char* lds_raw,
                          RelaxShared& sh, int64_t& flips, int64_t& logpos, uint64_t& hash,
                          uint64_t deadline) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int NT = blockDim.x, NW = NT >> 6;
  const int64_t n = I->n;
  const int l1s = I->l1_shift;
  const int nt1 = (int)((n + (1LL << l1s) - 1) >> l1s);
  const int nt2 = (nt1 + kL2Group - 1) / kL2Group;
  const int64_t nt0 = (n + 63) >> 6;
  const int per0 = 1 << (l1s - 6);  // per-64-row maxima in one tile
  const int seg = 1 << (l1s - 6);   // magnets per lane in a tile rescan
  RelaxLds L = carve(lds_raw, nt1, nt2);

  const int32_t D = I->D;
  const int32_t* __restrict__ colp = I->rcol;
  const double* __restrict__ Ap = I->rA;
  const double* __restrict__ Brp = I->rBr;
  const double* __restrict__ hkp = I->hk;
  int8_t* __restrict__ sp = I->s;
  double2* __restrict__ hp2 = I->h;
  double2* __restrict__ hd2 = I->hd;
  double* __restrict__ keyp = I->key;
  uint8_t* __restrict__ dirtyp = I->dirty;
  const int32_t mode = I->field_mode;
  const double pb = I->b, pc = I->c, ep = I->e_par, eq = I->e_perp;
  const int64_t max_flips = I->max_flips;

  // first level from the per-64-row maxima of the field phase (loads in
  // groups of 8, issued together)
  for (int e = tid; e < nt1; e += NT) {
    double bk = 0.0;
    uint32_t bi = 0;
    for (int u0 = 0; u0 < per0; u0 += 8) {
      double kk[8];
      uint32_t ki[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t f = (int64_t)e * per0 + u0 + u;
        const bool ok = u0 + u < per0 && f < nt0;
        kk[u] = ok ? I->t1key[f] : 0.0;
        ki[u] = ok ? I->t1idx[f] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (kk[u] > bk) {
          bk = kk[u];
          bi = ki[u];
        }
      }
    }
    L.l1k[e] = bk;
    L.l1i[e] = bi;
    L.l1flag[e] = 0;
    L.l1nk[e] = 0ull;
    L.l1ni[e] = ~0ull;
    L.l1resc[e] = 0;
  }
  if (tid == 0) {
    sh.nr = 0;
    sh.pfk = 0ull;
    sh.ruk = 0ull;
  }
  __syncthreads();
  for (int g = wave; g < nt2; g += NW) {
    const int e = g * kL2Group + lane;
    double k = (e < nt1) ? L.l1k[e] : 0.0;
    uint32_t pay = (e < nt1) ? L.l1i[e] : 0u;
    wave_argmax(k, pay);
    if (lane == 0) {
      L.l2k[g] = k;
      L.l2i[g] = pay;
      L.l2flag[g] = 0;
    }
  }
  __syncthreads();

  int status = 0;
  const int per2 = (nt2 + 63) >> 6;
  const int64_t flips0 = flips;
  // Row of the predicted next flip (the best magnet the last update pushed
  // over the astroid, the usual next flip of an avalanche), loaded while the
  // tree is brought up to date; used when the prediction holds.
  int64_t pf_j = -1;
  int32_t pf_c[2] = {-1, -1};
  double pf_a[2] = {0.0, 0.0}, pf_b[2] = {0.0, 0.0};

  // Up to kFlatTiles tiles the root reads the first level directly (at most
  // eight ascending tiles per lane) and the second level is not kept; only
  // in the tree-only kernel, whose registers allow it.
  const bool flat = kFlatOk && nt1 <= kFlatTiles;
  const int per1 = (nt1 + 63) >> 6;

  while (true) {
    if (wave == 0) {
      double bk = 0.0;
      uint32_t bp = 0;
      if (flat) {
        // the lane's tiles four at a time, each group's reads issued together
        for (int u0 = 0; u0 < per1; u0 += 4) {
          double kk[4];
          uint32_t ii[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = lane * per1 + u0 + u;
            const int ec = (u0 + u < per1 && e < nt1) ? e : 0;
            kk[u] = L.l1k[ec];
            ii[u] = L.l1i[ec];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = lane * per1 + u0 + u;
            if (u0 + u < per1 && e < nt1 && kk[u] > bk) {
              bk = kk[u];
              bp = ii[u];
            }
          }
        }
      } else {
        // second level of the groups the last flip touched (their flags; at
        // most kMaxL1Tiles / kL2Group = 32 groups, one per lane), then the root
        const bool gf = lane < nt2 && L.l2flag[lane] != 0;
        unsigned long long gbal = __ballot(gf);
        if (gf) L.l2flag[lane] = 0;
        while (gbal) {
          const int g = __ffsll(gbal) - 1;
          gbal &= gbal - 1ull;
          const int e = g * kL2Group + lane;
          double k = (e < nt1) ? L.l1k[e] : 0.0;
          uint32_t p2 = (e < nt1) ? L.l1i[e] : 0u;
          wave_argmax(k, p2);
          if (lane == 0) {
            L.l2k[g] = k;
            L.l2i[g] = p2;
          }
        }
        for (int u = 0; u < per2; ++u) {
          const int g = lane * per2 + u;
          if (g < nt2) {
            const double k = L.l2k[g];
            if (k > bk) {
              bk = k;
              bp = L.l2i[g];
            }
          }
        }
      }
      wave_argmax(bk, bp);
      if (lane == 0) {
        sh.key = bk;
        sh.pay = bp;
        sh.pause = (flips > flips0 && ((flips - flips0) & 15) == 0 && past(deadline)) ? 1 : 0;
      }
    }
    __syncthreads();
    const double top = sh.key;
    const uint32_t pay = sh.pay;
    if (!(top > 0.0)) break;
    if (sh.pause) {
      status = 1;
      break;
    }
    if (flips >= max_flips) {
      status = -5;
      break;
    }
    const int64_t j = pay & 0x7fffffffu;
    const int s_new = (pay & 0x80000000u) ? 1 : -1;
    if (tid == 0) {
      const uint64_t w = ((uint64_t)(uint32_t)t << 32) | (uint64_t)(uint32_t)j;
      hash = (hash ^ w) * 0x100000001b3ull;
      const int e = (int)(j >> l1s);
      L.l1resc[e] = 1;  // j was its tile's maximum
      L.l1flag[e] = 1;
    }
    ++logpos;
    ++flips;
    const double two = (s_new > 0) ? 2.0 : -2.0;
    // Update the neighbours.  A touched tile whose maximum was not among the
    // updated magnets, or kept at least its key, keeps that maximum unless an
    // update beats it, so it needs no rescan: the largest new key of the tile is found with LDS
    // atomics (positive doubles order like their bit patterns), then the
    // lowest index among the updates holding it.
    const bool incr = D <= 2 * NT;
    const bool hit = j == pf_j;
    // The predicted row's loads were issued before the last tile rescans,
    // whose loads the wavefront has waited for, so they are complete; using
    // the registers here makes that known, and no wait below is widened to
    // them.
    asm volatile("" ::"v"(pf_c[0]), "v"(pf_c[1]), "v"(pf_a[0]), "v"(pf_a[1]), "v"(pf_b[0]),
                 "v"(pf_b[1]));
    int u_i[2], u_e[2], u_s[2];
    double u_k[2];
    double tb_k = 0.0;  // this thread's best updated key, for the prediction
    uint32_t tb_i = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) u_i[h] = -1;
    for (int k = tid, h = 0; k < D; k += NT, ++h) {
      const int64_t sl = j * D + k;
      const bool pre = hit && h < 2;
      // the slot's column and couplings together (a padding slot holds -1
      // and zeros), then every load of the neighbour's state before any
      // store, so that each costs one round trip
      const int32_t i = pre ? pf_c[h & 1] : colp[sl];
      const double ca = pre ? pf_a[h & 1] : Ap[sl];
      const double cb = pre ? pf_b[h & 1] : Brp[sl];
      if (i >= 0) {
        const double2 hi = hp2[i];
        const double2 di = (mode == kFieldCarry) ? hd2[i] : make_double2(0.0, 0.0);
        const int si = sp[i];
        const double hki = hkp[i];
        const double da = two * ca;
        const double db = two * cb;
        const double hp = hi.x + da;
        const double hq = hi.y + db;
        const double kk = switching_key(si, hp, hq, hki, pb, pc, ep, eq);
        if (mode == kFieldCarry) {
          hd2[i] = make_double2(di.x + da, di.y + db);
        } else if (mode == kFieldDirty) {
          dirtyp[i] = 1;
        }
        hp2[i] = make_double2(hp, hq);
        keyp[i] = kk;
        const int e = (int)(i >> l1s);
        const double ek = L.l1k[e];
        const uint32_t ei = L.l1i[e];
        L.l1flag[e] = 1;
        if (!incr || (ek > 0.0 && (ei & 0x7fffffffu) == (uint32_t)i && kk < ek)) L.l1resc[e] = 1;
        if (kk > 0.0) atomicMax(&L.l1nk[e], (unsigned long long)__double_as_longlong(kk));
        if (kk > tb_k) {
          tb_k = kk;
          tb_i = (uint32_t)i;
        }
        if (h < 2) {
          u_i[h] = i;
          u_e[h] = e;
          u_s[h] = si;
          u_k[h] = kk;
        }
      }
    }
    // Runner-up hint, by the last wavefront when it updates no neighbour:
    // the best magnet of the tree outside j's tile (the other groups' maxima,
    // then the other tiles of j's group), the usual next flip when no update
    // beats it.  Read while the tree is unchanged since the root.
    if (wave == NW - 1 && D <= (NW - 1) * 64) {
      const int ej = (int)(j >> l1s), gj = ej / kL2Group;
      double rk = 0.0;
      uint32_t rp = 0;
      if (flat) {
        for (int u = 0; u < per1; ++u) {
          const int e = lane * per1 + u;
          if (e < nt1 && e != ej && L.l1k[e] > rk) {
            rk = L.l1k[e];
            rp = L.l1i[e];
          }
        }
      } else {
        for (int u = 0; u < per2; ++u) {
          const int g = lane * per2 + u;
          if (g < nt2 && g != gj && L.l2k[g] > rk) {
            rk = L.l2k[g];
            rp = L.l2i[g];
          }
        }
        const int e = gj * kL2Group + lane;
        if (e < nt1 && e != ej && L.l1k[e] > rk) {
          rk = L.l1k[e];
          rp = L.l1i[e];
        }
      }
      wave_argmax(rk, rp);
      if (lane == 0)
        sh.ruk = rk > 0.0 ? (((unsigned long long)__double_as_longlong(rk) & 0xffffffff00000000ull) |
                             (unsigned long long)(rp & 0x7fffffffu))
                          : 0ull;
    }
    // the flipped magnet's own stores, issued after the neighbour loads so
    // that waiting for those loads does not wait for these
    if (tid == 0) {
      sp[j] = (int8_t)s_new;
      keyp[j] = 0.0;
      if (logpos - 1 < I->log_cap) {
        I->log_t[logpos - 1] = (int32_t)t;
        I->log_j[logpos - 1] = (int32_t)j;
      }
    }
    wave_argmax(tb_k, tb_i);
    if (lane == 0 && tb_k > 0.0)
      atomicMax(&sh.pfk, ((unsigned long long)__double_as_longlong(tb_k) & 0xffffffff00000000ull) |
                             (unsigned long long)tb_i);
    __syncthreads();
    {
      // the next flip is probably the better of the best updated neighbour
      // and the runner-up (compared on the keys' high bits)
      const unsigned long long pk = sh.pfk > sh.ruk ? sh.pfk : sh.ruk;
      pf_j = pk ? (int64_t)(pk & 0xffffffffull) : -1;
      if (pf_j >= 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = tid + h * NT;
          if (k < D) {
            const int64_t sl = pf_j * D + k;
            pf_c[h] = colp[sl];
            pf_a[h] = Ap[sl];
            pf_b[h] = Brp[sl];
          }
        }
      }
    }
    if (incr) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (u_i[h] >= 0 && u_k[h] > 0.0 &&
            (unsigned long long)__double_as_longlong(u_k[h]) == L.l1nk[u_e[h]])
          atomicMin(&L.l1ni[u_e[h]], ((unsigned long long)u_i[h] << 1) | (u_s[h] < 0 ? 1ull : 0ull));
      }
    }
    __syncthreads();
    if (tid == 0) sh.pfk = 0ull;  // every thread has read it
    // touched tiles: a scan of the flags (nt1 <= kMaxL1Tiles), each tile's
    // state read at once
    for (int e = tid; e < nt1; e += NT) {
      if (!L.l1flag[e]) continue;
      if (L.l1resc[e]) {
        L.l1rlist[atomicAdd(&sh.nr, 1)] = e;
      } else {
        const unsigned long long nkb = L.l1nk[e];
        if (nkb != 0ull) {
          const double nk = __longlong_as_double((long long)nkb);
          const unsigned long long ni = L.l1ni[e];
          const uint32_t np = (uint32_t)(ni >> 1) | ((ni & 1ull) ? 0x80000000u : 0u);
          if (!(L.l1k[e] > 0.0) || better(nk, np, L.l1k[e], L.l1i[e])) {
            L.l1k[e] = nk;
            L.l1i[e] = np;
          }
        }
        L.l1flag[e] = 0;
        L.l2flag[e / kL2Group] = 1;
      }
      L.l1nk[e] = 0ull;
      L.l1ni[e] = ~0ull;
    }
    __syncthreads();
    const int nr = sh.nr;
    for (int u = wave; u < nr; u += NW) {
      const int e = L.l1rlist[u];
      const int64_t r0 = ((int64_t)e << l1s) + (int64_t)lane * seg;
      double bk = 0.0;
      uint32_t bp = 0;
      // the lane's segment in groups of 8, each group's loads issued together
      // (whole groups inside the arrays: four 16-byte key loads and one
      // 8-byte spin load, the group starting on a 64-byte boundary)
      for (int m0 = 0; m0 < seg; m0 += 8) {
        double kk[8];
        int ss[8];
        if (seg >= 8 && r0 + m0 + 8 <= n) {
          const double2* k2 = reinterpret_cast<const double2*>(keyp + r0 + m0);
          const uint64_t s8 = *reinterpret_cast<const uint64_t*>(sp + r0 + m0);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const double2 v = k2[m];
            kk[2 * m] = v.x;
            kk[2 * m + 1] = v.y;
          }
#pragma unroll
          for (int m = 0; m < 8; ++m) ss[m] = (int)(int8_t)(uint8_t)(s8 >> (8 * m));
        } else {
          // short segment or the array's end: every load issued at once, an
          // index past the segment replaced by magnet 0 and its key dropped
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const int64_t ii = r0 + m0 + m;
            const int64_t ic = (m0 + m < seg && ii < n) ? ii : 0;
            kk[m] = keyp[ic];
            ss[m] = sp[ic];
          }
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            if (!(m0 + m < seg && r0 + m0 + m < n)) {
              kk[m] = 0.0;
              ss[m] = 0;
            }
          }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          if (kk[m] > bk) {
            bk = kk[m];
            bp = (uint32_t)(r0 + m0 + m) | (ss[m] < 0 ? 0x80000000u : 0u);
          }
        }
      }
      wave_argmax(bk, bp);
      if (lane == 0) {
        L.l1k[e] = bk;
        L.l1i[e] = bp;
        L.l1flag[e] = 0;
        L.l1resc[e] = 0;
        L.l2flag[e / kL2Group] = 1;
      }
    }
    __syncthreads();
    if (tid == 0) sh.nr = 0;
  }
  return status;
}

// Per-64-row maxima of the stored keys -- the lowest level of the relax
// tree -- rebuilt by the whole workgroup, four 64-row groups per wavefront
// at a time (their loads issued together).
__device__ __forceinline__ void rebuild_t1(const InstDev* __restrict__ I) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
  const int64_t n = I->n, ng = (n + 63) >> 6;
  for (int64_t g0 = (int64_t)wave * 4; g0 < ng; g0 += (int64_t)NW * 4) {
    double k[4];
    uint32_t p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = ((g0 + u) << 6) + lane;
      k[u] = 0.0;
      p[u] = 0u;
      if (g0 + u < ng && i < n) {
        k[u] = I->key[i];
        p[u] = (uint32_t)i | (I->s[i] < 0 ? 0x80000000u : 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      wave_argmax(k[u], p[u]);
      if (lane == 0 && g0 + u < ng) {
        I->t1key[g0 + u] = k[u];
        I->t1idx[g0 + u] = p[u];
      }
    }
  }
  __syncthreads();
}

// Relax one instance at step t (Sec. II.H) and advance its run cursor.
// Steps that start with at least spec_min flippable magnets (and a degree
// that leaves room for batches) take the speculative path; the others the
// max tree; a speculative step whose batches stay small continues on the
// tree; a paused step resumes on the path it was on.  Both flip exactly the
// magnets, in exactly the order, of the one-at-a-time relax.
// kSpec false: the launch holds no instance that may speculate (every degree
// above kSpecMaxD, or a workgroup below 1024 threads), so the kernel carries
// the max tree alone and its registers are allocated for that path.
template <bool kSpec>
__device__ __forceinline__ int relax_step(const InstDev* __restrict__ I, RunDev* __restrict__ R, int64_t t,
                          unsigned char* lds_raw, RelaxShared& sh, SpecShared& ssh,
                          uint64_t deadline) {
  const int64_t ncand = __hip_atomic_load(I->ccount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t acc0 = R->step_acc;  // flips of step t before a pause
  int64_t flips = acc0;
  int64_t logpos = R->flips;
  uint64_t hash = R->hash;
  bool spec = kSpec && blockDim.x == 1024 &&
              (R->paused ? R->spec != 0 : (I->D <= kSpecMaxD && ncand >= I->spec_min));
  int status = 2;
  if ((int64_t)(uint32_t)ncand > I->ccap) {
    status = kPoolOverflow;  // cannot happen while every pass starts from an empty pool
  } else {
    if (kSpec && spec) status = relax_spec(I, t, lds_raw, ssh, ncand, flips, logpos, hash, deadline);
    if (status == 2) {
      if (kSpec && spec) rebuild_t1(I);  // the keys have moved since the field phase
      spec = false;
      status = relax_tree<!kSpec>(I, t, lds_raw, sh, flips, logpos, hash, deadline);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(I->ccount, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    R->flips += flips - acc0;
    R->flips_call += flips - acc0;
    R->hash = hash;
    if (status == 1) {
      R->step_acc = flips;
      R->paused = 1;
      R->spec = spec ? 1 : 0;
      R->active = 0;
    } else {
      if (t >= 0 && t < I->K && I->step_flips) I->step_flips[t] = (int32_t)flips;
      R->step_acc = 0;
      R->paused = 0;
      R->cur_step = t;
      R->t = t + 1;
      if (status != 0) R->status = status;
      R->active = (status == 0 && R->t < R->t_end) ? 1 : 0;
    }
  }
  __syncthreads();
  return status;
}

template <bool kSpec>
__global__ __launch_bounds__(64 * kMaxRelaxWaves) void k_relax(const InstDev* __restrict__ insts,
                                                              RunDev* __restrict__ runs) {
  RunDev* R = runs + blockIdx.x;
  // a relax paused at a burst deadline finishes its step here, its
  // structures rebuilt by the preceding field launch
  if (!R->active && !R->paused) return;
  extern __shared__ unsigned char lds_raw[];
  __shared__ RelaxShared sh;
  __shared__ SpecShared ssh;
  relax_step<kSpec>(insts + blockIdx.x, R, R->t, lds_raw, sh, ssh, 0);
}

// One workgroup per instance runs whole field steps -- its own field phase,
// wavefront by wavefront, then the relax -- through its own protocol, so
// instances never wait for each other between steps.  Stops after max_steps
// steps, at the end of the protocol, on ELOOP, or once budget_ticks of the
// constant-rate device clock have passed: checked between steps and inside
// the relax, which then pauses mid-step.  A paused instance finishes the
// step it stopped in first, its relax structures rebuilt (by the preceding
// field launch when first_ready); the flips it makes, and their order, are
// those of an uninterrupted relax.
__global__ __launch_bounds__(64 * kMaxRelaxWaves) void k_fused(const InstDev* __restrict__ insts,
                                                              RunDev* __restrict__ runs,
                                                              int64_t max_steps,
                                                              int64_t budget_ticks,
                                                              int32_t first_ready) {
  RunDev* R = runs + blockIdx.x;
  const bool paused = R->paused != 0;
  if (!R->active && !paused) return;
  const InstDev* I = insts + blockIdx.x;
  extern __shared__ unsigned char lds_raw[];
  __shared__ RelaxShared sh;
  __shared__ SpecShared ssh;
  __shared__ int go;
  const int wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
  const uint64_t t_start = wall_clock64();
  const uint64_t deadline = budget_ticks > 0 ? t_start + (uint64_t)budget_ticks : 0;
  bool ready = first_ready != 0;
  if (paused && !ready) {
    for (int64_t row0 = (int64_t)wave * 64; row0 < I->n; row0 += (int64_t)NW * 64)
      field_rows64_pool(I, row0, R->t, true);
    __syncthreads();
    ready = true;
  }
  for (int64_t k = 0; k < max_steps; ++k) {
    const int64_t t = R->t;
    if (!ready) {
      for (int64_t row0 = (int64_t)wave * 64; row0 < I->n; row0 += (int64_t)NW * 64)
        field_rows64_pool(I, row0, t);
      __syncthreads();
    }
    ready = false;
    if (relax_step<true>(I, R, t, lds_raw, sh, ssh, deadline) != 0) break;
    if (threadIdx.x == 0) go = (R->active && !past(deadline)) ? 1 : 0;
    __syncthreads();
    if (!go) break;
  }
}

// Run-cursor update, launched on the stream so it orders with the kernels
// (and can sit inside a captured graph).
__global__ void k_set_run(RunDev* R, int32_t* ccount, int64_t t, int64_t t_end, int32_t active,
                          int32_t reset_log, int64_t cur_step) {
  if (threadIdx.x != 0) return;
  if (ccount) *ccount = 0;  // the next field pass starts an empty candidate pool
  R->t = t;
  R->t_end = t_end;
  R->active = active;
  R->status = 0;
  R->flips_call = 0;
  R->paused = 0;
  R->step_acc = 0;
  if (reset_log) {
    R->flips = 0;
    R->hash = 0xcbf29ce484222325ull;
    R->cur_step = cur_step;
  }
}

// ------------------------------------------------------------ analysis
// Net magnetisation M = sum_i s_i mhat_i, the quantity a hysteresis loop
// plots (as M / M_S, M_S = n for unit moments).  Reduced in a fixed order,
// so the same spins give the same bits on every call: thread k of block b
// adds rows b*T + k, then every G*T rows, in ascending order; the block
// halves its sums in LDS; one block then halves the G block sums.
constexpr int kMagThreads = 256;
constexpr int kMagBlocks = 256;   // == kMagThreads: the final block takes one sum per thread

__device__ __forceinline__ void mag_halve(double* sx, double* sy) {
  for (int w = kMagThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sx[threadIdx.x] = sx[threadIdx.x] + sx[threadIdx.x + w];
      sy[threadIdx.x] = sy[threadIdx.x] + sy[threadIdx.x + w];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kMagThreads)
k_mag_partial(const int8_t* __restrict__ s, const double* __restrict__ mx,
              const double* __restrict__ my, int64_t n, double* __restrict__ part) {
  __shared__ double sx[kMagThreads], sy[kMagThreads];
  const int64_t stride = (int64_t)kMagBlocks * kMagThreads;
  double ax = 0.0, ay = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kMagThreads + threadIdx.x; i < n; i += stride) {
    const bool up = s[i] > 0;
    ax = ax + (up ? mx[i] : -mx[i]);
    ay = ay + (up ? my[i] : -my[i]);
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  mag_halve(sx, sy);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sx[0];
    part[2 * blockIdx.x + 1] = sy[0];
  }
}

__global__ void __launch_bounds__(kMagThreads)
k_mag_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sx[kMagThreads], sy[kMagThreads];
  sx[threadIdx.x] = part[2 * threadIdx.x];
  sy[threadIdx.x] = part[2 * threadIdx.x + 1];
  __syncthreads();
  mag_halve(sx, sy);
  if (threadIdx.x == 0) {
    out[0] = sx[0];
    out[1] = sy[0];
  }
}

static_assert(2 * kMagBlocks == kMagPartials, "block sums buffer");

// Net magnetisation of groups of magnets, e.g. the islands meeting at each
// vertex (the vertex maps of Sec. IV.B): group g sums s_i mhat_i over
// idx[ptr[g] .. ptr[g+1]) in that order, one thread per group.
__global__ void __launch_bounds__(256)
k_group_mag(const int8_t* __restrict__ s, const double* __restrict__ mx,
            const double* __restrict__ my, const int64_t* __restrict__ ptr,
            const int32_t* __restrict__ idx, int64_t ngroups, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  double ax = 0.0, ay = 0.0;
  for (int64_t e = ptr[g]; e < ptr[g + 1]; ++e) {
    const int32_t i = idx[e];
    const bool up = s[i] > 0;
    ax = ax + (up ? mx[i] : -mx[i]);
    ay = ay + (up ? my[i] : -my[i]);
  }
  out[2 * g] = ax;
  out[2 * g + 1] = ay;
}

// Spin-spin correlation by separation (Sec. IV.B): a pair (i, j) of
// neighbours correlates +1 when its dipolar energy -s_i s_j A_ij is at its
// minimum (s_i s_j A_ij > 0), -1 at its maximum, and 0 when the coupling
// vanishes (|A_ij| <= 1e-9 |alpha| / r^3, i.e. zero up to rounding).  Each
// pair counts once (j > i) in bin floor(r / w) of its distance r; pairs past
// the last bin are skipped.  The distance is formed with correctly rounded
// operations only, so the bin is the same as any IEEE evaluation of the
// same expression.  Sums and counts are integers, added per workgroup in
// LDS and then once per bin into the global totals.
__global__ void __launch_bounds__(256)
k_corr(const InstDev* __restrict__ I, const double* __restrict__ xy, double w, int32_t nbins,
       double abs_alpha, unsigned long long* __restrict__ sum, unsigned long long* __restrict__ cnt) {
  extern __shared__ int32_t lds_bins[];   // [2][nbins]
  int32_t* bs = lds_bins;
  int32_t* bc = lds_bins + nbins;
  for (int b = threadIdx.x; b < 2 * nbins; b += blockDim.x) lds_bins[b] = 0;
  __syncthreads();
  const int64_t n = I->n, D = I->D;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double xi = xy[2 * i], yi = xy[2 * i + 1];
    const int si = I->s[i];
    const int32_t L = I->len[i];
    // the sliced tables: slot k of 64 consecutive rows is contiguous, so
    // the lanes of a wavefront (consecutive rows) load it together
    for (int32_t k = 0; k < L; ++k) {
      const int64_t sl = slot_of(i, (int32_t)D, k);
      const int32_t j = I->col[sl];
      if (j <= i) continue;
      const double dx = __dsub_rn(xi, xy[2 * (int64_t)j]);
      const double dy = __dsub_rn(yi, xy[2 * (int64_t)j + 1]);
      const double r = __dsqrt_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)));
      const double q = floor(__ddiv_rn(r, w));
      if (!(q < (double)nbins)) continue;
      const int b = (int)q;
      const double a = I->A[sl];
      int c = 0;
      if (fabs(a) > 1e-9 * abs_alpha / (r * r * r)) c = ((si * I->s[j]) * (a > 0.0 ? 1 : -1) > 0) ? 1 : -1;
      atomicAdd(&bs[b], c);
      atomicAdd(&bc[b], 1);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    if (bc[b] != 0) {
      atomicAdd(&sum[b], (unsigned long long)(long long)bs[b]);
      atomicAdd(&cnt[b], (unsigned long long)bc[b]);
    }
  }
}

// Switching order of a flip log (Sec. IV.D): the log position of each
// magnet's first switch, and the twice-average rank of each magnet in that
// order.  Switched magnets have distinct first positions; a magnet that
// never switched is placed after all of them, so those magnets share the
// ranks S+1 .. n (S = switched magnets) and each gets their mean.  All of it
// is integer arithmetic: the results do not depend on the order of atomics.
constexpr int kRankBlock = 1024;  // log entries per block of the rank scan

__global__ void __launch_bounds__(256)
k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// pos[j] = smallest log position k with log_j[k] == j (pos preset to L).
__global__ void __launch_bounds__(256)
k_first_switch(const int32_t* __restrict__ log_j, int64_t L, unsigned long long* __restrict__ pos) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < L;
       k += (int64_t)gridDim.x * blockDim.x)
    atomicMin(&pos[log_j[k]], (unsigned long long)k);
}

// Log entry k is a first switch when pos[log_j[k]] == k.  Returns its
// exclusive rank among the first switches of this block's entries (uniform
// over the block after the call: wave totals in wtot[16]).
__device__ __forceinline__ int first_rank_in_block(const int32_t* __restrict__ log_j, int64_t L,
                                                   const unsigned long long* __restrict__ pos,
                                                   int* wtot, bool& first, int32_t& j,
                                                   int& block_total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t k = (int64_t)blockIdx.x * kRankBlock + tid;
  first = false;
  j = 0;
  if (k < L) {
    j = log_j[k];
    first = pos[j] == (unsigned long long)k;
  }
  const unsigned long long bal = __ballot(first);
  if (lane == 0) wtot[wave] = __popcll(bal);
  __syncthreads();
  int before = 0, tot = 0;
  for (int w = 0; w < kRankBlock / 64; ++w) {
    if (w < wave) before += wtot[w];
    tot += wtot[w];
  }
  block_total = tot;
  return before + __popcll(bal & ((1ull << lane) - 1ull));
}

__global__ void __launch_bounds__(kRankBlock)
k_first_count(const int32_t* __restrict__ log_j, int64_t L,
              const unsigned long long* __restrict__ pos, int64_t* __restrict__ cnt) {
  __shared__ int wtot[kRankBlock / 64];
  bool first;
  int32_t j;
  int tot;
  (void)first_rank_in_block(log_j, L, pos, wtot, first, j, tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

// Exclusive scan of the nb block counts by one workgroup (chunks of 1024
// with a running carry); total[0] = number of switched magnets.
__global__ void __launch_bounds__(kRankBlock)
k_scan_counts(const int64_t* __restrict__ cnt, int64_t nb, int64_t* __restrict__ off,
              int64_t* __restrict__ total) {
  __shared__ int64_t buf[kRankBlock];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += kRankBlock) {
    const int64_t v = (c0 + tid < nb) ? cnt[c0 + tid] : 0;
    buf[tid] = v;
    __syncthreads();
    for (int d = 1; d < kRankBlock; d <<= 1) {  // inclusive Hillis-Steele scan
      const int64_t add = tid >= d ? buf[tid - d] : 0;
      __syncthreads();
      buf[tid] += add;
      __syncthreads();
    }
    if (c0 + tid < nb) off[c0 + tid] = carry + buf[tid] - v;
    __syncthreads();
    if (tid == 0) carry += buf[kRankBlock - 1];
    __syncthreads();
  }
  if (tid == 0) total[0] = carry;
}

// Every magnet first gets the mean rank of the never-switched group,
// 2r = S + 1 + n; then each first switch overwrites its magnet's value.
__global__ void __launch_bounds__(256)
k_rank_rest(int64_t* __restrict__ r2, int64_t n, const int64_t* __restrict__ total) {
  const int64_t v = total[0] + 1 + n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r2[i] = v;
}

__global__ void __launch_bounds__(kRankBlock)
k_rank_switched(const int32_t* __restrict__ log_j, int64_t L,
                const unsigned long long* __restrict__ pos, const int64_t* __restrict__ off,
                int64_t* __restrict__ r2) {
  __shared__ int wtot[kRankBlock / 64];
  bool first;
  int32_t j;
  int tot;
  const int r = first_rank_in_block(log_j, L, pos, wtot, first, j, tot);
  if (first) r2[j] = 2 * (off[blockIdx.x] + r + 1);
}

// Pearson correlation of two rank vectors from exact sums: with u = 2r -
// (n + 1) per magnet, one block adds u_a u_b, u_a^2 and u_b^2 of its 256
// magnets into part[3 b .. 3 b + 2] (each |u| < n <= 2^27, so a block sum
// stays below 2^62).
constexpr int kCorrRankThreads = 256;

__global__ void __launch_bounds__(kCorrRankThreads)
k_rank_corr(const int64_t* __restrict__ r2a, const int64_t* __restrict__ r2b, int64_t n,
            long long* __restrict__ part) {
  __shared__ long long sab[kCorrRankThreads], saa[kCorrRankThreads], sbb[kCorrRankThreads];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kCorrRankThreads + tid;
  long long ua = 0, ub = 0;
  if (i < n) {
    ua = (long long)(r2a[i] - (n + 1));
    ub = (long long)(r2b[i] - (n + 1));
  }
  sab[tid] = ua * ub;
  saa[tid] = ua * ua;
  sbb[tid] = ub * ub;
  __syncthreads();
  for (int w = kCorrRankThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      sab[tid] += sab[tid + w];
      saa[tid] += saa[tid + w];
      sbb[tid] += sbb[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[3 * blockIdx.x] = sab[0];
    part[3 * blockIdx.x + 1] = saa[0];
    part[3 * blockIdx.x + 2] = sbb[0];
  }
}

// Exact totals of the nb block sums of k_rank_corr, one workgroup: each
// thread adds a strided subset of the blocks into 128-bit (low, high)
// accumulators, then the threads' accumulators are added pairwise in LDS.
// Integer sums, so the totals do not depend on the order (|total| < 2^81).
struct I128 {
  unsigned long long lo;
  long long hi;
};

__device__ inline I128 add128(I128 a, I128 b) {
  I128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

__device__ inline I128 widen(long long v) {
  I128 r;
  r.lo = (unsigned long long)v;
  r.hi = v < 0 ? -1 : 0;
  return r;
}

__global__ void __launch_bounds__(kCorrRankThreads)
k_rank_corr_total(const long long* __restrict__ part, int64_t nb, long long* __restrict__ tot) {
  __shared__ I128 acc[3][kCorrRankThreads];
  const int tid = threadIdx.x;
  I128 a[3] = {{0ull, 0}, {0ull, 0}, {0ull, 0}};
  for (int64_t b = tid; b < nb; b += kCorrRankThreads)
    for (int c = 0; c < 3; ++c) a[c] = add128(a[c], widen(part[3 * b + c]));
  for (int c = 0; c < 3; ++c) acc[c][tid] = a[c];
  __syncthreads();
  for (int w = kCorrRankThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int c = 0; c < 3; ++c) acc[c][tid] = add128(acc[c][tid], acc[c][tid + w]);
    __syncthreads();
  }
  if (tid < 3) {
    tot[2 * tid] = (long long)acc[tid][0].lo;
    tot[2 * tid + 1] = acc[tid][0].hi;
  }
}

// ------------------------------------------------------------ measurement
// Dependent-load latency: each of the first `lanes` lanes of one wavefront
// follows a chain of indices from its own start (each load's address comes
// from the previous load), `hops` times; lane 0 records the elapsed ticks of
// the device's constant-rate clock.  With 64 lanes a hop is one scattered
// 64-address gather, the unit of work of the relax's neighbour updates.  The
// chain is built and checked on the host to be one cycle over the buffer,
// so every load is in bounds however many hops are taken.
__global__ void k_chase(const int32_t* __restrict__ chain, const int32_t* __restrict__ starts,
                        int32_t lanes, int64_t hops, unsigned long long* __restrict__ out) {
  const int lane = threadIdx.x;
  if (blockIdx.x != 0 || lane >= lanes) return;
  int32_t p = starts[lane];
  const uint64_t t0 = wall_clock64();
  for (int64_t h = 0; h < hops; ++h) p = chain[p];
  const uint64_t t1 = wall_clock64();
  if (lane == 0) out[0] = t1 - t0;
  out[1 + lane] = (unsigned long long)p;  // keeps every chain live
}

}  // namespace

// ------------------------------------------------------------ launchers
void launch_chase(const int32_t* chain, const int32_t* starts, int32_t lanes, int64_t hops,
                  unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_chase, dim3(1), dim3(64), 0, st, chain, starts, lanes, hops, out);
}

int64_t switching_scratch_count(int64_t L) {
  const int64_t nb = std::max<int64_t>(1, (L + kRankBlock - 1) / kRankBlock);
  return 2 * nb + 1;
}

void launch_switching_ranks(const int32_t* log_j, int64_t L, int64_t n, unsigned long long* pos,
                            int64_t* r2, int64_t* scratch, hipStream_t st) {
  const int64_t nb = std::max<int64_t>(1, (L + kRankBlock - 1) / kRankBlock);
  const unsigned gn = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
  const unsigned gl = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (L + 255) / 256));
  int64_t* cnt = scratch;
  int64_t* off = scratch + nb;
  int64_t* total = scratch + 2 * nb;
  hipLaunchKernelGGL(k_fill_u64, dim3(gn), dim3(256), 0, st, pos, n, (unsigned long long)L);
  if (L > 0)
    hipLaunchKernelGGL(k_first_switch, dim3(gl), dim3(256), 0, st, log_j, L, pos);
  hipLaunchKernelGGL(k_first_count, dim3((unsigned)nb), dim3(kRankBlock), 0, st, log_j, L, pos,
                     cnt);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kRankBlock), 0, st, cnt, nb, off, total);
  hipLaunchKernelGGL(k_rank_rest, dim3(gn), dim3(256), 0, st, r2, n, total);
  hipLaunchKernelGGL(k_rank_switched, dim3((unsigned)nb), dim3(kRankBlock), 0, st, log_j, L, pos,
                     off, r2);
}

int64_t rank_corr_blocks(int64_t n) { return (n + kCorrRankThreads - 1) / kCorrRankThreads; }

void launch_rank_corr_total(const long long* part, int64_t nb, long long* tot, hipStream_t st) {
  hipLaunchKernelGGL(k_rank_corr_total, dim3(1), dim3(kCorrRankThreads), 0, st, part, nb, tot);
}

// ------------------------------------------------------------ static scratch
// Scratch of the allocation-free switching-order comparison: one array per
// GPU for the life of the process.  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress, per device.
namespace {

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t kRhoRankBytes = align256(8 * (size_t)kStaticRhoMaxN);
constexpr size_t kRhoTmpBytes =
    align256(8 * (size_t)(2 * ((kStaticRhoMaxLog + kRankBlock - 1) / kRankBlock) + 1));
constexpr size_t kRhoPartBytes =
    align256(8 * 3 * (size_t)((kStaticRhoMaxN + kCorrRankThreads - 1) / kCorrRankThreads));
constexpr size_t kRhoTotBytes = align256(8 * 6);
constexpr size_t kScratchBytes = 4 * kRhoRankBytes + 2 * kRhoTmpBytes + kRhoPartBytes + kRhoTotBytes;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxScratchDevices] = {};

}  // namespace

size_t static_scratch_bytes() { return kScratchBytes; }

StaticRhoScratch carve_static_rho(unsigned char* base) {
  StaticRhoScratch S;
  size_t off = 0;
  for (int k = 0; k < 2; ++k) {
    S.pos[k] = reinterpret_cast<unsigned long long*>(base + off);
    off += kRhoRankBytes;
    S.r2[k] = reinterpret_cast<int64_t*>(base + off);
    off += kRhoRankBytes;
  }
  for (int k = 0; k < 2; ++k) {
    S.tmp[k] = reinterpret_cast<int64_t*>(base + off);
    off += kRhoTmpBytes;
  }
  S.part = reinterpret_cast<long long*>(base + off);
  off += kRhoPartBytes;
  S.tot = reinterpret_cast<long long*>(base + off);
  return S;
}

hipError_t static_scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

void launch_rank_correlation(const int64_t* r2a, const int64_t* r2b, int64_t n, long long* part,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_rank_corr, dim3((unsigned)rank_corr_blocks(n)), dim3(kCorrRankThreads), 0,
                     st, r2a, r2b, n, part);
}

void launch_correlation(const InstDev* inst, int64_t n, const double* xy, double w,
                        int32_t nbins, double abs_alpha, uint64_t* sum, uint64_t* cnt,
                        hipStream_t st) {
  const int64_t blocks = std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_corr, dim3((unsigned)blocks), dim3(256), 2 * nbins * sizeof(int32_t), st,
                     inst, xy, w, nbins, abs_alpha,
                     reinterpret_cast<unsigned long long*>(sum),
                     reinterpret_cast<unsigned long long*>(cnt));
}

void launch_group_magnetization(const int8_t* s, const double* mx, const double* my,
                                const int64_t* ptr, const int32_t* idx, int64_t ngroups,
                                double* out, hipStream_t st) {
  const int64_t blocks = (ngroups + 255) / 256;
  hipLaunchKernelGGL(k_group_mag, dim3((unsigned)blocks), dim3(256), 0, st, s, mx, my, ptr, idx,
                     ngroups, out);
}

void launch_magnetization(const int8_t* s, const double* mx, const double* my, int64_t n,
                          double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mag_partial, dim3(kMagBlocks), dim3(kMagThreads), 0, st, s, mx, my, n,
                     part);
  hipLaunchKernelGGL(k_mag_final, dim3(1), dim3(kMagThreads), 0, st, part, out);
}

void launch_draw_hk(double* hk, int64_t n, double mean, double k, uint64_t seed, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_draw_hk, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, hk, n, mean, k,
                     seed);
}

void launch_neighbour_count(const double* x, const double* y, const int32_t* cellx,
                            const int32_t* celly, const int32_t* cell_start,
                            const int32_t* cell_members, int64_t n, int64_t gx, int64_t gy,
                            double cut2, int32_t* len, int32_t* dup_flag, hipStream_t st) {
  const int bs = 256;
  const int64_t nb = (n + bs - 1) / bs;
  hipLaunchKernelGGL(k_nb_count, dim3((unsigned)nb), dim3(bs), 0, st, x, y, cellx, celly,
                     cell_start, cell_members, n, gx, gy, cut2, len, dup_flag);
}

void launch_neighbour_fill(const double* x, const double* y, const double* mx, const double* my,
                           const int32_t* cellx, const int32_t* celly, const int32_t* cell_start,
                           const int32_t* cell_members, int64_t n, int64_t gx, int64_t gy,
                           double cut2, double alpha, int32_t D, int32_t* col, double* A,
                           double* B, int32_t* rcol, double* rA, double* rBr,
                           hipStream_t st) {
  const int bs = 128;
  const int64_t nb = (n + bs - 1) / bs;
  hipLaunchKernelGGL(k_nb_fill, dim3((unsigned)nb), dim3(bs), 0, st, x, y, mx, my, cellx, celly,
                     cell_start, cell_members, n, gx, gy, cut2, alpha, D, col, A, B, rcol, rA,
                     rBr);
}

void launch_field(const InstDev* insts, RunDev* runs, const int32_t* blk_inst,
                  const int32_t* blk_row0, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_field, dim3((unsigned)nblocks), dim3(kFieldBlock), 0, st, insts, runs,
                     blk_inst, blk_row0);
}

void launch_field_hd(const InstDev* inst, RunDev* run, int64_t n, int32_t rows, int32_t nch,
                     hipStream_t st) {
  const int64_t nsl = (n + 63) / 64;
  if (rows == 0 && nch > 0 && nsl < kHdSplitSlices) {
    hipLaunchKernelGGL(k_field_hd_part, dim3((unsigned)(nsl * nch)), dim3(512), 0, st, inst, run);
    hipLaunchKernelGGL(k_field_hd_comb, dim3((unsigned)((nsl + 3) / 4)), dim3(256), 0, st, inst,
                       run);
    return;
  }
  // rows per workgroup: by default the largest that still gives the device
  // about four workgroups per compute unit, at least 8
  const int R = rows ? rows
                     : nsl >= 1024 ? 64 : 2 * nsl >= 1024 ? 32 : 4 * nsl >= 1024 ? 16 : 8;
  const unsigned blocks = (unsigned)(((nsl + 7) / 8) * 8 * (64 / R));
  switch (R) {
    case 64:
      hipLaunchKernelGGL(k_field_hd<64>, dim3(blocks), dim3(512), 0, st, inst, run);
      break;
    case 32:
      hipLaunchKernelGGL(k_field_hd<32>, dim3(blocks), dim3(256), 0, st, inst, run);
      break;
    case 16:
      hipLaunchKernelGGL(k_field_hd<16>, dim3(blocks), dim3(128), 0, st, inst, run);
      break;
    default:
      hipLaunchKernelGGL(k_field_hd<8>, dim3(blocks), dim3(64), 0, st, inst, run);
      break;
  }
  if (R < 64)
    hipLaunchKernelGGL(k_slice_max, dim3((unsigned)((nsl + 3) / 4)), dim3(256), 0, st, inst, run);
}

void launch_relax(const InstDev* insts, RunDev* runs, int32_t count, int32_t waves,
                  size_t lds_bytes, bool tree_only, hipStream_t st) {
  if (count <= 0) return;
  if (tree_only)
    hipLaunchKernelGGL(k_relax<false>, dim3((unsigned)count), dim3(64 * waves), lds_bytes, st,
                       insts, runs);
  else
    hipLaunchKernelGGL(k_relax<true>, dim3((unsigned)count), dim3(64 * waves), lds_bytes, st,
                       insts, runs);
}

void launch_fused(const InstDev* insts, RunDev* runs, int32_t count, int32_t waves,
                  size_t lds_bytes, int64_t max_steps, int64_t budget_ticks,
                  int32_t first_ready, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fused, dim3((unsigned)count), dim3(64 * waves), lds_bytes, st, insts, runs,
                     max_steps, budget_ticks, first_ready);
}

void launch_set_run(RunDev* run, int32_t* ccount, int64_t t, int64_t t_end, int32_t active,
                    int32_t reset_log, int64_t cur_step, hipStream_t st) {
  hipLaunchKernelGGL(k_set_run, dim3(1), dim3(64), 0, st, run, ccount, t, t_end, active,
                     reset_log, cur_step);
}

int32_t relax_l1_shift(int64_t n) {
  int32_t s = 6;
  while (((n + (1LL << s) - 1) >> s) > kMaxL1Tiles) ++s;
  return s;
}

size_t relax_lds_bytes(int64_t n, int32_t l1_shift) {
  // one relax path runs per step, so the two share the space
  const size_t a = relax_tree_lds_bytes(n, l1_shift), b = spec_lds_bytes();
  return a > b ? a : b;
}

hipError_t configure_kernels() {
  // the relax kernels take more than 64 KB of dynamic LDS
  const int bytes = (int)relax_lds_bytes((int64_t)kMaxL1Tiles << 6, 6);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_relax<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_relax<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

}  // namespace asi
