// Internal device-side data layout shared by the kernels and the host runtime
// of the spin-ice library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

// Pointers to device memory held in the instance descriptor.  In the
// kernels' device pass they carry the global address space, so accesses
// through them compile to global loads and stores (a scalar base plus a
// vector offset, counted by the vector-memory counter only) instead of flat
// ones, whose completion every wait for an LDS access would also await.
// Elsewhere (host code, and the runtime's device pass, which holds no
// kernels) they are plain pointers; the layout is the same.
#if defined(__HIP_DEVICE_COMPILE__) && defined(ASI_KERNELS_UNIT)
#define ASI_GLOBAL __attribute__((address_space(1)))
#else
#define ASI_GLOBAL
#endif

namespace asi {

// Rows per neighbour-table slice: one row per lane of a wavefront.
constexpr int kSlice = 64;
// Rows per block of the grid-wide field pass (4 wavefronts).
constexpr int kFieldBlock = 256;
// Most first-level tiles the relax keeps in LDS.  A tile covers 2^l1_shift
// consecutive magnets (at least 64).
constexpr int kMaxL1Tiles = 2048;
// First-level tiles per second-level group (one per lane).
constexpr int kL2Group = 64;
// Max-tree relax: up to this many tiles the root reads the first level
// directly (eight tiles per lane) instead of a second level.
constexpr int kFlatTiles = 512;
// Largest relax workgroup.
constexpr int kMaxRelaxWaves = 16;
// Above this degree a speculative batch holds too few members to beat the
// max tree, so the relax never speculates.
constexpr int kSpecMaxD = 128;

// How the dipolar sum of a row is obtained at the start of a field step.
enum FieldMode : int32_t {
  kFieldCarry = 0,  // gathered once, then carried across steps by the flip deltas
  kFieldDirty = 1,  // re-gathered (canonical order) when a neighbour flipped
  kFieldFull = 2,   // re-gathered (canonical order) for every row every step
};

// Per-instance tables and state; device pointers.  One entry per instance
// in a device array, so a single launch can serve many instances.
struct InstDev {
  int64_t n;              // magnets
  int32_t D;              // padded row length of the neighbour tables
  int32_t l1_shift;       // log2 of the first-level tile size of the relax tree
  // Neighbour tables, sliced for the field pass (one row per lane): slot k
  // of row i lives at ((i / 64) * D + k) * 64 + (i % 64);  col == -1 pads a
  // row.
  const ASI_GLOBAL int32_t* len;     // [n] neighbours of each row
  const ASI_GLOBAL int32_t* col;     // neighbour index j (ascending within a row)
  const ASI_GLOBAL double* A;        // mhat_i    . c_ij  (symmetric: A_ij == A_ji)
  const ASI_GLOBAL double* B;        // mhatperp_i. c_ij  (field at row i from j)
  // The same rows row-major for the relax, which walks one row at a time
  // (a wavefront reads consecutive slots): slot k of row i at i * D + k.
  const ASI_GLOBAL int32_t* rcol;    // neighbour index j, -1 pads
  const ASI_GLOBAL double* rA;       // A_ij
  const ASI_GLOBAL double* rBr;      // mhatperp_j. c_ji  (field at neighbour j from row i)
  const ASI_GLOBAL double* mx;       // [n] easy axis mhat_i = (mx, my)
  const ASI_GLOBAL double* my;
  const ASI_GLOBAL double* hk;       // [n] coercive field h_k^(i)
  double b, c;            // astroid width parameters
  double e_par, e_perp;   // astroid exponents 2/gamma and 2/beta
  double sigma;           // thermal std
  const ASI_GLOBAL double* sigma_t;  // [K] thermal std of each step (replaces sigma), or null
  uint64_t seed;          // thermal Philox key
  const ASI_GLOBAL double* H;        // [K][2] applied field per step
  int64_t K;
  const ASI_GLOBAL double2* hloc;    // [hloc_k][n] per-magnet external field (x, y), or null
  int64_t hloc_k;         // 1: the same field at every step; else one per step (== K)
  // travelling-wave local field evaluated in the pass: wave_amp * sin(wave_ph[i]
  // - wave_w * t) along (wave_ex, wave_ey); wave_ph null when none
  const ASI_GLOBAL double* wave_ph;  // [n] 2 pi (k . r_i) + phase0
  double wave_amp, wave_w, wave_ex, wave_ey;
  int32_t field_mode;     // FieldMode
  int32_t pad0;
  // mutable state
  ASI_GLOBAL int8_t* s;              // [n] spins
  ASI_GLOBAL uint8_t* dirty;         // [n] row's dipolar sum must be gathered at the next step
  // Field pairs (x: easy axis, y: hard axis) kept together, so the relax
  // reads or writes a magnet's pair with one 16-byte access.
  ASI_GLOBAL double2* hd;            // [n] dipolar field (gathered, plus flip deltas)
  ASI_GLOBAL double2* h;             // [n] total field (dipolar + applied + thermal)
  ASI_GLOBAL double* key;            // [n] Eq. 5 LHS if flippable, else 0
  ASI_GLOBAL double* t1key;          // [ceil(n/64)] per-64-row maximum key
  ASI_GLOBAL uint32_t* t1idx;        //   its index, bit 31 set when that spin is -1
  // Per-chunk dipolar sums of the high-degree pass split over its 64-slot
  // chunks: [nch][n] (easy, hard); null and nch == 0 when not allocated
  ASI_GLOBAL double2* part;
  int32_t nch;
  int32_t pad1;
  ASI_GLOBAL int32_t* log_t;         // flip log
  ASI_GLOBAL int32_t* log_j;
  int64_t log_cap;
  ASI_GLOBAL int32_t* step_flips;    // [K] flips of each step (may be null)
  int64_t max_flips;      // per relax
  // candidate pool of the speculative relax: the field phase appends every
  // flippable magnet as (key, index | sign bit, version) to buffer 0
  ASI_GLOBAL uint32_t* ver;          // [n] version of each magnet's key
  ASI_GLOBAL uint32_t* cpay[2];      // [ccap] pool buffers
  ASI_GLOBAL double* ckey[2];
  ASI_GLOBAL uint32_t* cver[2];
  ASI_GLOBAL int32_t* ccount;        // entries in buffer 0 (field phase appends)
  int64_t ccap;
  int64_t spec_min;       // flippable magnets at step start to go speculative
  double spec_switch;     // mean batch below which a speculative step goes on the tree
};

// Per-instance run cursor, device-resident so repeated launches (and
// captured graphs) advance each instance through its own protocol.
struct RunDev {
  int64_t t;          // step the next field pass evaluates (-1: no field)
  int64_t t_end;      // run stops before this step
  int32_t active;     // instance takes part in the next launch
  int32_t status;     // 0, ASI_ELOOP or kPoolOverflow
  int64_t flips;      // flips since create / set_state
  int64_t flips_call; // flips since the host last cleared it
  uint64_t hash;      // running flip-log hash
  int64_t cur_step;   // last relaxed step
  // A relax stopped at a deadline part-way through step t leaves active = 0
  // and paused = 1; the relax structures are rebuilt from the key array and
  // step t continues on the same relax path (spec: speculative).  step_acc
  // counts the flips step t has made so far.
  int32_t paused;
  int32_t spec;
  int64_t step_acc;
};

// Coercive fields drawn from the disorder distribution (asi_params.hk == NULL).
void launch_draw_hk(double* hk, int64_t n, double mean, double k, uint64_t seed, hipStream_t st);
// Net magnetisation sum_i s_i mhat_i of n magnets into out[2]; part holds
// kMagPartials doubles of block sums.  Fixed reduction order.
constexpr int kMagPartials = 2 * 256;
void launch_magnetization(const int8_t* s, const double* mx, const double* my, int64_t n,
                          double* part, double* out, hipStream_t st);
// Net magnetisation of each CSR group of magnets (ptr [ngroups+1], idx on
// the device, indices validated by the caller) into out[ngroups][2].
void launch_group_magnetization(const int8_t* s, const double* mx, const double* my,
                                const int64_t* ptr, const int32_t* idx, int64_t ngroups,
                                double* out, hipStream_t st);
// Spin-spin correlation sums and pair counts per distance bin (two's
// complement sums) over the instance's neighbour pairs; xy is on the device.
constexpr int kCorrMaxBins = 4096;
void launch_correlation(const InstDev* inst, int64_t n, const double* xy, double w,
                        int32_t nbins, double abs_alpha, uint64_t* sum, uint64_t* cnt,
                        hipStream_t st);
// Switching order of a flip log of L entries over n magnets (Sec. IV.D):
// pos[j] = log position of magnet j's first switch (L if none), r2[j] =
// twice its average rank in that order (integers; never-switched magnets
// tie).  scratch: switching_scratch_count(L) int64 on the device.
int64_t switching_scratch_count(int64_t L);
void launch_switching_ranks(const int32_t* log_j, int64_t L, int64_t n, unsigned long long* pos,
                            int64_t* r2, int64_t* scratch, hipStream_t st);
// Exact partial sums of u_a u_b, u_a^2, u_b^2 (u = r2 - (n + 1)) per block
// of magnets into part[3 * rank_corr_blocks(n)]; requires n <= 2^27.
constexpr int64_t kRankCorrMaxN = (int64_t)1 << 27;
int64_t rank_corr_blocks(int64_t n);
void launch_rank_correlation(const int64_t* r2a, const int64_t* r2b, int64_t n, long long* part,
                             hipStream_t st);
// Exact totals of the rank_correlation block sums (Sab, Saa, Sbb) into
// tot[6] as 128-bit two's complement (low, high) pairs; one workgroup.
void launch_rank_corr_total(const long long* part, int64_t nb, long long* tot, hipStream_t st);
// Allocation-free comparison of switching orders: size limits and the
// regions of the library's static device scratch (one copy per GPU, held
// until the process ends), carved from its device address.
constexpr int64_t kStaticRhoMaxN = (int64_t)1 << 20;    // magnets per instance
constexpr int64_t kStaticRhoMaxLog = (int64_t)1 << 24;  // flips in each flip log
struct StaticRhoScratch {
  unsigned long long* pos[2];  // [kStaticRhoMaxN] first-switch positions of a, b
  int64_t* r2[2];              // [kStaticRhoMaxN] twice-average ranks of a, b
  int64_t* tmp[2];             // [switching_scratch_count(kStaticRhoMaxLog)] of a, b
  long long* part;             // [3 rank_corr_blocks(kStaticRhoMaxN)]
  long long* tot;              // [6]
};
size_t static_scratch_bytes();
StaticRhoScratch carve_static_rho(unsigned char* base);
// Device address of the static scratch on the current device: looked up
// with hipGetSymbolAddress on the first call on each device (with that
// device current), then taken from a per-device table.
hipError_t static_scratch_address(unsigned char** out);
// Pointer chase (measurement): lanes 0 .. lanes-1 (<= 64) of one wavefront
// each take `hops` dependent loads along chain from starts[lane]; out[0] =
// elapsed device-clock ticks, out[1 + lane] = each lane's last index.
void launch_chase(const int32_t* chain, const int32_t* starts, int32_t lanes, int64_t hops,
                  unsigned long long* out, hipStream_t st);
void launch_neighbour_count(const double* x, const double* y, const int32_t* cellx,
                            const int32_t* celly, const int32_t* cell_start,
                            const int32_t* cell_members, int64_t n, int64_t gx, int64_t gy,
                            double cut2, int32_t* len, int32_t* dup_flag, hipStream_t st);
void launch_neighbour_fill(const double* x, const double* y, const double* mx, const double* my,
                           const int32_t* cellx, const int32_t* celly, const int32_t* cell_start,
                           const int32_t* cell_members, int64_t n, int64_t gx, int64_t gy,
                           double cut2, double alpha, int32_t D, int32_t* col, double* A,
                           double* B, int32_t* rcol, double* rA, double* rBr, hipStream_t st);
// Degree from which a single instance's full-field pass (every row
// gathered) uses one workgroup per 64-row slice instead of one lane per row.
constexpr int kHdMinD = 128;
// Full-field pass of one instance of degree >= kHdMinD (field_mode full),
// `rows` rows per workgroup (8, 16, 32 or 64; 0: chosen by the size).  With
// rows == 0, nch > 0 (the per-chunk sums allocated) and fewer than
// kHdSplitSlices slices, the pass is split over the 64-slot chunks: a
// workgroup per (slice, chunk), then a combine pass over the rows.
void launch_field_hd(const InstDev* inst, RunDev* run, int64_t n, int32_t rows, int32_t nch,
                     hipStream_t st);
// Below this many 64-row slices the high-degree pass is split over chunks
// (even 8 rows per workgroup then leave the device mostly idle while each
// workgroup walks its chunks; above it the split's extra partial-sum
// traffic and combine pass cost more than they save).
constexpr int64_t kHdSplitSlices = 256;
// Grid-wide field pass for every active instance of the table; rebuilds the
// relax structures of every paused one.
void launch_field(const InstDev* insts, RunDev* runs, const int32_t* blk_inst,
                  const int32_t* blk_row0, int64_t nblocks, hipStream_t st);
// One workgroup per instance: relax the current step.  tree_only when no
// instance of the launch may speculate (see relax_may_speculate): the kernel
// then holds the max tree alone.
void launch_relax(const InstDev* insts, RunDev* runs, int32_t count, int32_t waves,
                  size_t lds_bytes, bool tree_only, hipStream_t st);
// Whether an instance of degree D relaxed by workgroups of `waves` wavefronts
// may take the speculative path (it needs the full 16-wavefront workgroup).
inline bool relax_may_speculate(int32_t D, int32_t waves) {
  return waves == kMaxRelaxWaves && D <= kSpecMaxD;
}
// One workgroup per instance: up to max_steps whole steps (field phase and
// relax) per instance.  With budget_ticks > 0 a workgroup stops once that many ticks of the
// device's constant-rate clock have passed: between steps, or inside a relax
// (which then pauses, see RunDev).  With first_ready a field launch has just
// computed each active instance's fields and rebuilt each paused one's relax
// structures.
void launch_fused(const InstDev* insts, RunDev* runs, int32_t count, int32_t waves,
                  size_t lds_bytes, int64_t max_steps, int64_t budget_ticks,
                  int32_t first_ready, hipStream_t st);
// Run-cursor update on the stream; with ccount, also empties the
// instance's candidate pool.
void launch_set_run(RunDev* run, int32_t* ccount, int64_t t, int64_t t_end, int32_t active,
                    int32_t reset_log, int64_t cur_step, hipStream_t st);
// RunDev::status of a step whose candidate pool overflowed its capacity
// (an internal error: the host reports ASI_EDEVICE).
constexpr int32_t kPoolOverflow = -3;
// Dynamic LDS of the relax and fused kernels for an instance of n magnets.
size_t relax_lds_bytes(int64_t n, int32_t l1_shift);
int32_t relax_l1_shift(int64_t n);
// Raise the dynamic-LDS limit of the relax kernels (call once per process).
hipError_t configure_kernels();

}  // namespace asi
