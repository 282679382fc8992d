// Oracle, tier 1: plain single-threaded FP64 CPU implementation of the
// flatspin dipole model (Jensen et al., "flatspin: A Large-Scale Artificial
// Spin Ice Simulator", Sec. II).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the package smoke check and the CPU
// baseline leg of the benchmark use it.  It shares no code, header, table or
// helper with the HIP library.
//
// Build: g++ -O2 -ffp-contract=off -fPIC -shared relax.cpp -o liborc.so
// (no FMA contraction: every product and sum rounds on its own).
//
// What it computes, in the paper's order:
//   Eq. 1   m_i = s_i * mhat_i,  mhat_i = (cos th_i, sin th_i)
//   Eq. 3   h_dip_i = alpha * sum_{j in N(i)} [3 r (m_j . r)/|r|^5 - m_j/|r|^3],
//           r = r_i - r_j, N(i) = { j != i : |r_i - r_j| <= d } (Sec. II.C:
//           neighbourhood in lattice units; inclusive, tested as
//           dx^2 + dy^2 <= (d + 1e-9)^2), summed in ascending j.
//   Eq. 2   h_i = h_dip_i + h_ext_i + h_th_i         (xy frame)
//           h_ext_i = H[t] + hloc_i(t): the global field of step t plus the
//           magnet's own local field (Sec. II.D), static or one per step
//           h_par = h_i . mhat_i, h_perp = h_i . mhat_perp_i,
//           mhat_perp_i = (-sin th_i, cos th_i)       (Sec. II.F, Fig. 2)
//   Eq. 5   L_i = (|h_par|/(b hk_i))^(2/gamma) + (|h_perp|/(c hk_i))^(2/beta)
//           c = +inf drops the h_perp term; with b = 1, gamma = 2 the test is
//           then the parallel-only criterion -s_i h_par > hk_i (Sec. IV.C)
//   Eq. 6   flippable <=> s_i h_par_i < 0  and  L_i > 1
//   Sec. II.H  repeat { flip argmax_i L_i over flippable (ties: lowest i);
//              recompute fields } until none; then next field step.  The
//              external and thermal fields are constant during a relax.
//   Sec. II.E  thermal field: two orthogonal (x, y) components, each
//              N(0, sigma_th^2) (or N(0, sigma_t[t]^2) under an annealing
//              schedule, Sec. IV.B), drawn once per magnet per step from
//              Philox4x32-10 (Salmon et al., SC'11) keyed (seed_lo, seed_hi)
//              with counter (i, t, 0, 0), mapped by Box-Muller.
//
// After a flip of j only the fields of j's neighbours change, so exactly those
// rows are re-summed from Eq. 3 (full row, ascending j) -- the same values a
// complete re-evaluation of every field would give.  The per-edge bracket of
// Eq. 3 for a unit source moment is cached (a value cache, not a reordering).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <set>
#include <utility>
#include <vector>

namespace {

// ---------------------------------------------------------------- Philox
struct U32x4 { uint32_t v[4]; };

inline void mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

// Philox4x32 with 10 rounds: each round multiplies counter words 0 and 2 by
// the two round multipliers and mixes the high halves with words 1, 3 and the
// key; the key is advanced by the two Weyl constants between rounds.
U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo(M0, c.v[0], &hi0, &lo0);
    mulhilo(M1, c.v[2], &hi1, &lo1);
    U32x4 o;
    o.v[0] = hi1 ^ c.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ c.v[3] ^ k1;
    o.v[3] = lo0;
    c = o;
  }
  return c;
}

// Two standard normals for (seed, counter) by the Box-Muller transform.
void normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t tag,
                 double* z0, double* z1) {
  U32x4 c = {{c0, c1, tag, 0u}};
  U32x4 o = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  uint64_t a = ((((uint64_t)o.v[0]) << 32) | o.v[1]) >> 11;
  uint64_t bb = ((((uint64_t)o.v[2]) << 32) | o.v[3]) >> 11;
  const double two_m53 = 1.0 / 9007199254740992.0;  // 2^-53
  double u1 = (double)(a + 1) * two_m53;            // (0, 1]
  double u2 = (double)bb * two_m53;                 // [0, 1)
  const double two_pi = 6.283185307179586;
  double rad = std::sqrt(-2.0 * std::log(u1));
  double ang = two_pi * u2;
  *z0 = rad * std::cos(ang);
  *z1 = rad * std::sin(ang);
}

// ---------------------------------------------------------------- model
struct Model {
  int64_t n = 0;
  std::vector<double> x, y, mx, my, px, py, hk;
  double alpha = 0, d = 0, b = 1, c = 1, beta = 3, gamma = 3;
  double sigma_th = 0;
  uint64_t seed = 0;
  std::vector<int64_t> nb_ptr;      // [n+1]
  std::vector<int32_t> nb_idx;      // ascending j per row
  std::vector<double> gx, gy;       // Eq. 3 bracket, unit source moment
  std::vector<double> gabs;         // alpha * sum_j |g_ij| per row (scale)
  std::vector<int8_t> s;
  std::vector<double> hdx, hdy;     // alpha * sum_j s_j g_ij
  std::vector<double> sig_t;        // [K] thermal std per step (annealing), or empty
  std::vector<double> loc;          // [loc_k][n][2] local external field
  int64_t loc_k = 0;                // 0 none, 1 static, else one per step
};

void build_neighbours(Model& M) {
  const int64_t n = M.n;
  const double cut = M.d + 1e-9;
  const double cut2 = cut * cut;
  double xmin = M.x[0], xmax = M.x[0], ymin = M.y[0], ymax = M.y[0];
  for (int64_t i = 1; i < n; ++i) {
    xmin = std::min(xmin, M.x[i]); xmax = std::max(xmax, M.x[i]);
    ymin = std::min(ymin, M.y[i]); ymax = std::max(ymax, M.y[i]);
  }
  double cs = cut;
  if (cs < 1e-6) cs = 1e-6;
  // keep the grid modest; larger cells only cost more candidate tests
  while ((xmax - xmin) / cs > 4096.0 || (ymax - ymin) / cs > 4096.0) cs *= 2.0;
  const int64_t gx = (int64_t)std::floor((xmax - xmin) / cs) + 1;
  const int64_t gy = (int64_t)std::floor((ymax - ymin) / cs) + 1;
  std::vector<int64_t> cell(n);
  std::vector<int64_t> start(gx * gy + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = (int64_t)std::floor((M.x[i] - xmin) / cs);
    int64_t cy = (int64_t)std::floor((M.y[i] - ymin) / cs);
    cx = std::min(std::max(cx, (int64_t)0), gx - 1);
    cy = std::min(std::max(cy, (int64_t)0), gy - 1);
    cell[i] = cy * gx + cx;
    start[cell[i] + 1]++;
  }
  for (int64_t k = 0; k < gx * gy; ++k) start[k + 1] += start[k];
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  std::vector<int32_t> members(n);
  for (int64_t i = 0; i < n; ++i) members[fill[cell[i]]++] = (int32_t)i;

  M.nb_ptr.assign(n + 1, 0);
  M.nb_idx.clear();
  std::vector<int32_t> row;
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    int64_t cx = cell[i] % gx, cy = cell[i] / gx;
    for (int64_t yy = std::max<int64_t>(0, cy - 1); yy <= std::min(gy - 1, cy + 1); ++yy)
      for (int64_t xx = std::max<int64_t>(0, cx - 1); xx <= std::min(gx - 1, cx + 1); ++xx) {
        int64_t k = yy * gx + xx;
        for (int64_t p = start[k]; p < start[k + 1]; ++p) {
          int32_t j = members[p];
          if (j == i) continue;
          double dx = M.x[i] - M.x[j];
          double dy = M.y[i] - M.y[j];
          if (dx * dx + dy * dy <= cut2) row.push_back(j);
        }
      }
    std::sort(row.begin(), row.end());
    M.nb_idx.insert(M.nb_idx.end(), row.begin(), row.end());
    M.nb_ptr[i + 1] = (int64_t)M.nb_idx.size();
  }
}

void build_brackets(Model& M) {
  const int64_t E = (int64_t)M.nb_idx.size();
  M.gx.resize(E); M.gy.resize(E);
  M.gabs.assign(M.n, 0.0);
  for (int64_t i = 0; i < M.n; ++i) {
    double acc = 0.0;
    for (int64_t e = M.nb_ptr[i]; e < M.nb_ptr[i + 1]; ++e) {
      int32_t j = M.nb_idx[e];
      // Eq. 3 with a unit source moment mhat_j at r_j, observed at r_i
      double rx = M.x[i] - M.x[j];
      double ry = M.y[i] - M.y[j];
      double r2 = rx * rx + ry * ry;
      double r = std::sqrt(r2);
      double r3 = r2 * r;
      double r5 = r3 * r2;
      double mr = M.mx[j] * rx + M.my[j] * ry;
      M.gx[e] = 3.0 * rx * mr / r5 - M.mx[j] / r3;
      M.gy[e] = 3.0 * ry * mr / r5 - M.my[j] / r3;
      acc += std::fabs(M.gx[e]) + std::fabs(M.gy[e]);
    }
    M.gabs[i] = M.alpha * acc;
  }
}

// Eq. 3 for one row, from the current spins, ascending j.
void dipolar_row(Model& M, int64_t i) {
  double sx = 0.0, sy = 0.0;
  for (int64_t e = M.nb_ptr[i]; e < M.nb_ptr[i + 1]; ++e) {
    double sj = (double)M.s[M.nb_idx[e]];
    sx += sj * M.gx[e];
    sy += sj * M.gy[e];
  }
  M.hdx[i] = M.alpha * sx;
  M.hdy[i] = M.alpha * sy;
}

struct StepFields {
  double Hx = 0, Hy = 0;
  const double* loc = nullptr;   // [n][2] local field of this step, or none
  std::vector<double> thx, thy;  // empty when sigma_th == 0
};

// Local external field of step t (none before the first step).
const double* local_for_step(const Model& M, int64_t t) {
  if (M.loc_k == 0 || t < 0) return nullptr;
  const int64_t k = (M.loc_k == 1) ? 0 : t;
  return &M.loc[(size_t)(2 * k * M.n)];
}

// Step t < 0 is the state before the first field step: no thermal draw.
// With a schedule, step t uses its own standard deviation sig_t[t].
void thermal_for_step(const Model& M, int64_t t, StepFields& F) {
  const double sigma = (M.sig_t.empty() || t < 0) ? M.sigma_th : M.sig_t[(size_t)t];
  if (sigma == 0.0 || t < 0) { F.thx.clear(); F.thy.clear(); return; }
  F.thx.resize(M.n); F.thy.resize(M.n);
  for (int64_t i = 0; i < M.n; ++i) {
    double z0, z1;
    normal_pair(M.seed, (uint32_t)i, (uint32_t)t, 0u, &z0, &z1);
    F.thx[i] = sigma * z0;
    F.thy[i] = sigma * z1;
  }
}

struct Eval { double hpar, hperp, L; bool flip; };

// Eq. 2 then the switching test of Eq. 5 and Eq. 6 for magnet i.
Eval evaluate(const Model& M, const StepFields& F, int64_t i) {
  double hx = M.hdx[i] + F.Hx;
  double hy = M.hdy[i] + F.Hy;
  if (F.loc) { hx = hx + F.loc[2 * i]; hy = hy + F.loc[2 * i + 1]; }
  if (!F.thx.empty()) { hx = hx + F.thx[i]; hy = hy + F.thy[i]; }
  Eval ev;
  ev.hpar = hx * M.mx[i] + hy * M.my[i];
  ev.hperp = hx * M.px[i] + hy * M.py[i];
  ev.L = 0.0;
  ev.flip = false;
  if ((double)M.s[i] * ev.hpar < 0.0) {
    double a = std::fabs(ev.hpar) / (M.b * M.hk[i]);
    double q = std::fabs(ev.hperp) / (M.c * M.hk[i]);
    ev.L = std::pow(a, 2.0 / M.gamma) + std::pow(q, 2.0 / M.beta);
    ev.flip = ev.L > 1.0;
  }
  return ev;
}

struct Gaps {
  double min_top2_rel = INFINITY;   // (L1 - L2) / L1 at each pick
  double min_thresh_rel = INFINITY; // |L - 1| over right-direction evaluations
  double min_par_rel = INFINITY;    // |h_par| / scale over all evaluations
};

inline void note(Gaps& G, const Model& M, const StepFields& F, int64_t i, const Eval& ev) {
  double scale = M.gabs[i] + std::hypot(F.Hx, F.Hy);
  if (F.loc) scale += std::hypot(F.loc[2 * i], F.loc[2 * i + 1]);
  if (!F.thx.empty()) scale += std::hypot(F.thx[i], F.thy[i]);
  if (scale > 0.0) G.min_par_rel = std::min(G.min_par_rel, std::fabs(ev.hpar) / scale);
  if ((double)M.s[i] * ev.hpar < 0.0) G.min_thresh_rel = std::min(G.min_thresh_rel, std::fabs(ev.L - 1.0));
}

}  // namespace

extern "C" {

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  U32x4 c = {{ctr[0], ctr[1], ctr[2], ctr[3]}};
  U32x4 o = philox4x32_10(c, key[0], key[1]);
  for (int k = 0; k < 4; ++k) out[k] = o.v[k];
}

// Sec. II.G disorder: h_k^(i) = mean + (k * mean) * z_i with z_i the first
// normal of counter (i, 0, 1, 0); draws below 1e-12 * mean are raised to it.
void orc_disorder_hk(int64_t n, double mean, double k, uint64_t seed, double* out) {
  const double sd = k * mean;
  const double lo = 1e-12 * mean;
  for (int64_t i = 0; i < n; ++i) {
    double z0, z1;
    normal_pair(seed, (uint32_t)i, 0u, 1u, &z0, &z1);
    const double h = mean + sd * z0;
    out[i] = h < lo ? lo : h;
  }
}

void orc_normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t tag, double* z) {
  normal_pair(seed, c0, c1, tag, &z[0], &z[1]);
}

void* orc_create(int64_t n, const double* xy, const double* theta, const double* hk,
                 double alpha, double d, double b, double c, double beta, double gamma,
                 double sigma_th, uint64_t seed) {
  if (n < 1) return nullptr;
  Model* M = new Model();
  M->n = n;
  M->x.resize(n); M->y.resize(n); M->mx.resize(n); M->my.resize(n);
  M->px.resize(n); M->py.resize(n); M->hk.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    M->x[i] = xy[2 * i]; M->y[i] = xy[2 * i + 1];
    M->mx[i] = std::cos(theta[i]); M->my[i] = std::sin(theta[i]);
    M->px[i] = -M->my[i]; M->py[i] = M->mx[i];
    M->hk[i] = hk[i];
  }
  M->alpha = alpha; M->d = d; M->b = b; M->c = c; M->beta = beta; M->gamma = gamma;
  M->sigma_th = sigma_th; M->seed = seed;
  build_neighbours(*M);
  build_brackets(*M);
  M->s.assign(n, 1);
  M->hdx.assign(n, 0.0); M->hdy.assign(n, 0.0);
  return M;
}

void orc_destroy(void* h) { delete static_cast<Model*>(h); }

int64_t orc_num_edges(void* h) { return (int64_t)static_cast<Model*>(h)->nb_idx.size(); }

void orc_neighbours(void* h, int64_t* ptr, int32_t* idx) {
  Model& M = *static_cast<Model*>(h);
  std::memcpy(ptr, M.nb_ptr.data(), sizeof(int64_t) * (M.n + 1));
  if (!M.nb_idx.empty()) std::memcpy(idx, M.nb_idx.data(), sizeof(int32_t) * M.nb_idx.size());
}

void orc_set_spins(void* h, const int8_t* s) {
  Model& M = *static_cast<Model*>(h);
  for (int64_t i = 0; i < M.n; ++i) M.s[i] = s[i] >= 0 ? 1 : -1;
  for (int64_t i = 0; i < M.n; ++i) dipolar_row(M, i);
}

// Local external field (Sec. II.D): loc[k][n][2] for k < loc_k; loc_k = 1
// applies slab 0 at every step, loc_k > 1 gives step t slab t; 0 removes it.
void orc_set_local_field(void* h, int64_t loc_k, const double* loc) {
  Model& M = *static_cast<Model*>(h);
  M.loc_k = loc_k;
  M.loc.assign(loc, loc + (size_t)(2 * loc_k * M.n));
}

// Thermal schedule (annealing): sigma[t] for steps 0..K-1 replaces sigma_th;
// K = 0 returns to sigma_th.
void orc_set_thermal_schedule(void* h, int64_t K, const double* sigma) {
  Model& M = *static_cast<Model*>(h);
  M.sig_t.assign(sigma, sigma + (size_t)K);
}

void orc_get_spins(void* h, int8_t* s) {
  Model& M = *static_cast<Model*>(h);
  std::memcpy(s, M.s.data(), M.n);
}

// Total fields (h_par, h_perp) at step t under applied field H (2 doubles),
// for the current spins (plus the local field of step t, if set); `scale`
// gets the summand scale alpha*sum|g| + |H| + |hloc| + |h_th| per magnet.
// With a local series, t must be below its length.  Any output may be NULL.
void orc_fields(void* h, const double* H, int64_t t, double* hpar, double* hperp,
                double* hdx, double* hdy, double* scale) {
  Model& M = *static_cast<Model*>(h);
  StepFields F;
  F.Hx = H[0]; F.Hy = H[1];
  F.loc = local_for_step(M, t);
  thermal_for_step(M, t, F);
  for (int64_t i = 0; i < M.n; ++i) {
    Eval ev = evaluate(M, F, i);
    if (hpar) hpar[i] = ev.hpar;
    if (hperp) hperp[i] = ev.hperp;
    if (hdx) hdx[i] = M.hdx[i];
    if (hdy) hdy[i] = M.hdy[i];
    if (scale) {
      double sc = M.gabs[i] + std::hypot(F.Hx, F.Hy);
      if (F.loc) sc += std::hypot(F.loc[2 * i], F.loc[2 * i + 1]);
      if (!F.thx.empty()) sc += std::hypot(F.thx[i], F.thy[i]);
      scale[i] = sc;
    }
  }
}

// Checksum of a flip log, independent of the library's: FNV-1a over one
// 64-bit word per flip, (uint32 step << 32 | uint32 index): h = (h ^ w) *
// 1099511628211 mod 2^64, starting from 14695981039346656037.
inline uint64_t fnv_fold(uint64_t h, int64_t t, int32_t j) {
  const uint64_t w = ((uint64_t)(uint32_t)t << 32) | (uint64_t)(uint32_t)j;
  return (h ^ w) * 1099511628211ull;
}

// Run field steps t_begin .. t_end-1 of the protocol H[K][2] (Sec. II.H).
// Returns 0, or -5 when a step exceeds max_flips_per_step (0: no cap).
// Flip log entries beyond log_cap are counted but not stored.
// gaps (may be NULL) receives {min_top2_rel, min_thresh_rel, min_par_rel};
// step_top2 (may be NULL) the smallest top-two relative gap of each step
// (+inf where a step never had two candidates).  fnv (may be NULL) is
// folded with every flip, stored or not.
int orc_run(void* h, int64_t K, const double* H, int64_t t_begin, int64_t t_end,
            int32_t* log_t, int32_t* log_j, int64_t log_cap, int64_t* n_flips,
            int32_t* flips_per_step, double* gaps, int64_t max_flips_per_step,
            uint64_t* fnv, double* step_top2) {
  Model& M = *static_cast<Model*>(h);
  Gaps G;
  uint64_t hsum = fnv ? *fnv : 0ull;
  int64_t count = 0;
  int status = 0;
  std::vector<double> L(M.n, 0.0);
  std::vector<char> in_set(M.n, 0);
  StepFields F;
  for (int64_t t = t_begin; t < t_end && status == 0; ++t) {
    if (t < 0 || t >= K || (M.loc_k > 1 && t >= M.loc_k) ||
        (!M.sig_t.empty() && t >= (int64_t)M.sig_t.size())) { status = -1; break; }
    F.Hx = H[2 * t]; F.Hy = H[2 * t + 1];
    F.loc = local_for_step(M, t);
    thermal_for_step(M, t, F);
    std::set<std::pair<double, int32_t>> cand;   // (-L_i, i): begin() = max L, min i
    for (int64_t i = 0; i < M.n; ++i) {
      Eval ev = evaluate(M, F, i);
      note(G, M, F, i, ev);
      in_set[i] = ev.flip;
      L[i] = ev.L;
      if (ev.flip) cand.insert(std::make_pair(-ev.L, (int32_t)i));
    }
    int64_t step_flips = 0;
    double step_gap = INFINITY;
    while (!cand.empty()) {
      auto top = cand.begin();
      int32_t j = top->second;
      if (cand.size() > 1) {
        auto nxt = std::next(top);
        double l1 = -top->first, l2 = -nxt->first;
        step_gap = std::min(step_gap, (l1 - l2) / l1);
      }
      cand.erase(top);
      in_set[j] = 0;
      if (max_flips_per_step > 0 && step_flips >= max_flips_per_step) { status = -5; break; }
      M.s[j] = (int8_t)(-M.s[j]);
      if (count < log_cap) { log_t[count] = (int32_t)t; log_j[count] = j; }
      hsum = fnv_fold(hsum, t, j);
      ++count;
      ++step_flips;
      // fields change exactly on j's neighbours: re-sum them from Eq. 3
      for (int64_t e = M.nb_ptr[j]; e < M.nb_ptr[j + 1]; ++e) dipolar_row(M, M.nb_idx[e]);
      // re-test j and its neighbours (j's own field is unchanged)
      auto retest = [&](int64_t i) {
        Eval ev = evaluate(M, F, i);
        note(G, M, F, i, ev);
        if (in_set[i]) cand.erase(std::make_pair(-L[i], (int32_t)i));
        in_set[i] = ev.flip;
        L[i] = ev.L;
        if (ev.flip) cand.insert(std::make_pair(-ev.L, (int32_t)i));
      };
      retest(j);
      for (int64_t e = M.nb_ptr[j]; e < M.nb_ptr[j + 1]; ++e) retest(M.nb_idx[e]);
    }
    if (flips_per_step) flips_per_step[t - t_begin] = (int32_t)step_flips;
    if (step_top2) step_top2[t - t_begin] = step_gap;
    G.min_top2_rel = std::min(G.min_top2_rel, step_gap);
  }
  if (n_flips) *n_flips = count;
  if (fnv) *fnv = hsum;
  if (gaps) { gaps[0] = G.min_top2_rel; gaps[1] = G.min_thresh_rel; gaps[2] = G.min_par_rel; }
  return status;
}

}  // extern "C"
