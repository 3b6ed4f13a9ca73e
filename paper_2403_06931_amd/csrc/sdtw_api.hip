// sdtw_api.hip -- host side of libsdtw.so: argument validation, workspace
// layout, tile-variant table and kernel launches behind the C ABI declared in
// include/sdtw.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "sdtw.h"
#include "sdtw_argmin.hpp"
#include "sdtw_bwd.hpp"
#include "sdtw_fwd.hpp"
#include "sdtw_quant.hpp"
#include "sdtw_setup.hpp"
#include "sdtw_variant.hpp"
#include "sdtw_znorm.hpp"

#include "sdtw_variants.inc"
SDTW_VARIANTS(SDTW_DECLARE_VARIANT)

// Workspace of the allocation-free forward (sdtw_forward_noalloc): a fixed
// array of the library's device code.  Every GPU that loads the library
// holds its own copy, at its own address, until the process ends.  In host
// code this name is only a handle for hipGetSymbolAddress: kernels and copies
// take the device address that call returns (scratch_address()).
static __device__ __align__(256) unsigned char scratch[SDTW_NOALLOC_SCRATCH_BYTES];

namespace {

using sdtw::FwdParams;

constexpr size_t kAlign = 256;
constexpr int kCkptQuantum = 16;   // ckpt_every must be a multiple of every tile width

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

using sdtw::Variant;

const Variant& variant(int i) {
#define SDTW_VARIANT_ENTRY(i, R, T, W, KS, XL) sdtw_variant_entry_##i(),
  static const Variant table[] = {SDTW_VARIANTS(SDTW_VARIANT_ENTRY)};
#undef SDTW_VARIANT_ENTRY
  return table[i];
}

int variant_count() {
#define SDTW_COUNT_ONE(i, R, T, W, KS, XL) +1
  return 0 SDTW_VARIANTS(SDTW_COUNT_ONE);
#undef SDTW_COUNT_ONE
}

// ------------------------------------------------------------------ checks

bool lens_ok(const int32_t* h_lens, int32_t batch, int64_t* total, int32_t* nmax) {
  if (h_lens == nullptr || batch < 1) return false;
  int64_t s = 0;
  int32_t mx = 0;
  for (int32_t b = 0; b < batch; ++b) {
    if (h_lens[b] < 1) return false;
    s += h_lens[b];
    mx = std::max(mx, h_lens[b]);
  }
  if (total) *total = s;
  if (nmax) *nmax = mx;
  return true;
}

bool ref_ok(int64_t ref_len) { return ref_len >= 1 && ref_len <= SDTW_MAX_REF_LEN; }

int64_t row_stride_floats(int64_t ref_len) { return (int64_t)align_up((size_t)ref_len, 64); }

// Batches up to this size let each workgroup sum the lengths before its
// query instead of running the offset-table kernel first.
constexpr int32_t kInKernelOffsetBatch = 16384;

// Forward workspace: offset and slot tables (used above kInKernelOffsetBatch
// queries), the persistent form's work counter and processing order, and the
// row buffer that carries the last row of a row pass to the next pass.
struct FwdLayout {
  size_t offsets, ranks, queue, order, rowbuf, total;
  int64_t slots;
};

FwdLayout fwd_layout(int32_t batch, int64_t ref_len, int32_t flags, int64_t slots) {
  FwdLayout L{};
  size_t at = 0;
  L.offsets = at;
  at = align_up(at + sizeof(int64_t) * ((size_t)batch + 1), kAlign);
  L.ranks = at;
  at = align_up(at + sizeof(int32_t) * (size_t)batch, kAlign);
  L.queue = at;
  at = align_up(at + sizeof(int32_t) * 4, kAlign);
  L.order = at;
  at = align_up(at + ((flags & SDTW_F_PERSISTENT) ? sizeof(int32_t) * (size_t)batch : 0), kAlign);
  L.rowbuf = at;
  L.slots = slots;
  at = align_up(at + sizeof(float) * (size_t)slots * (size_t)row_stride_floats(ref_len), kAlign);
  L.total = at;
  return L;
}

// uint8-code forward: the plain forward's workspace, then the codes of the
// queries and of the reference, the per-chunk extremes and the codebook.
struct U8Layout {
  FwdLayout fwd;
  size_t qcodes, rcodes, part, book, total;
  int nparts;
};

U8Layout u8_layout(int32_t batch, int64_t total_rows, int64_t ref_len) {
  U8Layout L{};
  L.fwd = fwd_layout(batch, ref_len, 0, batch);   // one row-buffer slot per query
  size_t at = L.fwd.total;
  L.qcodes = at;
  at = align_up(at + (size_t)total_rows, kAlign);
  L.rcodes = at;
  at = align_up(at + (size_t)ref_len, kAlign);
  L.nparts = (int)((ref_len + sdtw::kQChunk - 1) / sdtw::kQChunk);
  L.part = at;
  at = align_up(at + sizeof(float2) * (size_t)L.nparts, kAlign);
  L.book = at;
  at = align_up(at + sizeof(sdtw::QBook), kAlign);
  L.total = at;
  return L;
}

constexpr int kU8Codes = 3;             // forward_impl's kind for the code DP

// Forward flags: checkpoints, persistent launch and the persistent grid's
// wavefronts per SIMD (0 = the default, 2; at most 8).
constexpr int32_t kFwdFlags = SDTW_F_CHECKPOINT | SDTW_F_PERSISTENT | SDTW_F_WAVES_MASK;

bool fwd_flags_ok(int32_t flags) {
  return (flags & ~kFwdFlags) == 0 && ((flags & SDTW_F_WAVES_MASK) >> SDTW_F_WAVES_SHIFT) <= 8;
}

// Persistent grid: the requested wavefronts per SIMD (default two), at most
// one workgroup per query.
// Teams (of W wavefronts) in the persistent grid, and its workgroups of
// persistent_teams(W) teams each.
int64_t persistent_teams_for(const Variant& v, int32_t batch, int cus, int32_t flags) {
  const int wps = (flags & SDTW_F_WAVES_MASK) >> SDTW_F_WAVES_SHIFT;
  const int64_t waves_per_cu = 4LL * (wps > 0 ? wps : 2);
  return std::max<int64_t>(1, std::min<int64_t>(batch, (int64_t)cus * waves_per_cu / v.W));
}

int64_t persistent_grid_for(const Variant& v, int32_t batch, int cus, int32_t flags) {
  const int64_t tpw = sdtw::persistent_teams(v.W);
  return (persistent_teams_for(v, batch, cus, flags) + tpw - 1) / tpw;
}

// Row-buffer slots a forward launch of variant v needs: the plain launch
// gives one to each query longer than one pass of the tile (64 R W rows),
// indexed by its rank among those queries; the persistent launch one to each
// team of its grid (every team of every workgroup), if any query needs a
// second pass.  Queries that fit in one pass never touch the row buffer.
int64_t fwd_slots(const Variant& v, const int32_t* h_lens, int32_t batch, int32_t flags,
                  int cus) {
  const int64_t rows = 64LL * v.R * v.W;
  int64_t multi = 0;
  for (int32_t b = 0; b < batch; ++b) multi += h_lens[b] > rows ? 1 : 0;
  if (flags & SDTW_F_PERSISTENT)
    return multi > 0 ? persistent_grid_for(v, batch, cus, flags) * sdtw::persistent_teams(v.W)
                     : 0;
  return multi;
}

// Rows of the row-checkpoint region: query b's rows kRowCkpt*k < len_b
// (k >= 1) sit at region rows offset(b)/kRowCkpt + k - 1, which never
// overlap the next query's (the floor of a sum bounds the sum of floors).
static_assert(sdtw::kRowCkpt == SDTW_ROW_CKPT_EVERY, "row-checkpoint spacing");
int64_t row_ckpt_rows(int64_t total_len) { return total_len / sdtw::kRowCkpt; }

int64_t n_ckpt_of(int64_t ref_len, int32_t every) {
  if (every < 1) return -1;
  return (ref_len + every - 1) / every - 1;
}

// Estimated relative time of a variant on this batch (used when the caller
// lets the library choose): padded cells x VALU instructions per cell over
// the issue rate the launch can sustain.  gfx950 dual-issues VALU from two
// ready wavefronts of a SIMD, so the rate grows with resident wavefronts per
// SIMD (factors measured on 512 x 2,000 vs 100,000 and 256 x 1,000 vs 50,000).
double variant_cost(const Variant& v, const int32_t* h_lens, int32_t batch, int64_t ref_len,
                    int cus) {
  const int64_t rows = 64LL * v.R * v.W;
  const int64_t ntiles = (ref_len + v.T - 1) / v.T;
  // pipeline fill: each lane lags its neighbour by one step (both exchange
  // forms), each wavefront the previous one by KS steps more
  const int64_t skew = (64LL * v.W - 1) + (v.W - 1) * v.KS;
  double cells = 0;
  for (int32_t b = 0; b < batch; ++b) {
    const int64_t passes = (h_lens[b] + rows - 1) / rows;
    cells += (double)passes * rows * (double)(ntiles + skew) * v.T;
  }
  // per-cell VALU work: 4 cell ops and about 8 per-step instructions; the
  // DPP form adds one move per row-block column, and its DPP moves cost
  // dual issue (about 10 % measured at R = 8)
  const double per_cell =
      (4.0 + 8.0 / (v.R * v.T) + (v.XL ? 0.0 : 1.0 / v.R)) * (v.XL ? 1.0 : 1.1);
  // wavefronts per SIMD: the batch's, capped by the workgroups one CU holds
  // (160 KiB of LDS, 32 wavefronts)
  constexpr int kLdsPerCu = 160 * 1024;
  const int wg_per_cu = std::max(1, std::min(kLdsPerCu / std::max(1, v.lds_bytes), 32 / v.W));
  const double wps = std::min((double)batch * v.W / (4.0 * cus), wg_per_cu * v.W / 4.0);
  static const double kIssue[] = {0.0, 0.55, 0.75, 0.85, 1.0};   // by min(4, ceil(wps))
  const int slot = wps <= 0 ? 1 : (wps >= 4 ? 4 : (int)(wps + 0.999));
  const double rate = kIssue[slot] * std::min(1.0, wps / slot);
  return cells * per_cell / rate;
}

// Compute units of the current device (read once per device; a CPX or other
// partition mode shows fewer than the full chip's 256).
int device_cus() {
  constexpr int kMaxDevices = 64;
  static int cached[kMaxDevices] = {0};
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev >= 0 && dev < kMaxDevices && cached[dev] > 0) return cached[dev];
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
    v = 256;
  if (dev >= 0 && dev < kMaxDevices) cached[dev] = v;
  return v;
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current; nullptr if the lookup fails.
void* scratch_address() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {nullptr};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return nullptr;
    addr[dev] = p;
  }
  return addr[dev];
}

int pick_variant(const int32_t* h_lens, int32_t batch, int64_t ref_len, int32_t flags, int cus) {
  (void)flags;
  int best = 0;
  double best_cost = 0;
  for (int i = 0; i < variant_count(); ++i) {
    const double c = variant_cost(variant(i), h_lens, batch, ref_len, cus);
    if (i == 0 || c < best_cost) {
      best = i;
      best_cost = c;
    }
  }
  return best;
}

// Backward: direction codes of `slots` blocks per query are held per round,
// in two buffers (the walk of one round overlaps the recompute of the next);
// both are kept under kBwdCodeBudget bytes where the batch allows, with at
// least one block per round.
constexpr size_t kBwdCodeBudget = size_t(2) << 30;
// Round kernels from this one on recompute their blocks as row bands.  The
// first two recomputes (rounds 0 and 1: every query's first blocks, then
// those of nearly every query, since round 1's are started before round 0's
// walk ends) are bound by issue slots, where bands would only add pipeline
// fill and more wavefronts beside the walkers: whole blocks there.
constexpr int kFirstBandedKernel = 1;
// Band height, a multiple of the row-checkpoint spacing.  (On 256 x 1,000
// vs 50,000, bands of 512 rows in the first banded kernel and 256 after it
// measured 1.58 ms per backward, 512 throughout 1.61-1.62 ms, 256
// throughout 1.52 ms: the shorter latency outweighs the extra pipeline
// fill.)
constexpr int kBandRows = 256;
static_assert(kBandRows % sdtw::kRowCkpt == 0, "bands start on row checkpoints");

struct BwdLayout {
  size_t offsets, state, lo, row_lo, row_hi, part, codes, total;
  int64_t code_half;          // words per code buffer
  int32_t nseg, slots, rounds;
};

// with_grad = false (sdtw_align): no per-query reference partials.
BwdLayout bwd_layout(int32_t batch, int64_t total_len, int64_t ref_len, int32_t ckpt_every,
                     bool with_grad = true) {
  BwdLayout L{};
  L.nseg = (ckpt_every + sdtw::kDirSeg - 1) / sdtw::kDirSeg;
  const size_t words_per_slot =
      (size_t)L.nseg * sdtw::kWave * ((size_t)total_len + (size_t)(sdtw::kWave - 1) * batch);
  const size_t bytes_per_slot = words_per_slot * sizeof(uint32_t);
  const int64_t nblk = (ref_len + ckpt_every - 1) / ckpt_every;
  int64_t slots = (int64_t)(kBwdCodeBudget / (2 * bytes_per_slot));
  slots = std::max<int64_t>(1, std::min<int64_t>({slots, sdtw::kBwdMaxSlots, nblk}));
  L.slots = (int32_t)slots;
  L.rounds = (int32_t)((nblk + slots - 1) / slots);
  size_t at = 0;
  L.offsets = at;
  at = align_up(at + sizeof(int64_t) * ((size_t)batch + 1), kAlign);
  L.state = at;
  at = align_up(at + sizeof(int32_t) * 4 * (size_t)batch, kAlign);
  L.lo = at;
  at = align_up(at + sizeof(int32_t) * (size_t)batch, kAlign);
  L.row_lo = at;
  at = align_up(at + sizeof(int32_t) * (size_t)total_len, kAlign);
  L.row_hi = at;
  at = align_up(at + sizeof(int32_t) * (size_t)total_len, kAlign);
  L.part = at;
  if (with_grad)
    at = align_up(at + sizeof(float) * (size_t)batch * (size_t)row_stride_floats(ref_len),
                  kAlign);
  L.codes = at;
  L.code_half = (int64_t)(words_per_slot * (size_t)slots);
  at = align_up(at + 2 * bytes_per_slot * (size_t)slots, kAlign);
  L.total = at;
  return L;
}

// Normaliser workspace: element and chunk offsets, chunk -> series map and
// the binary64 chunk partials.
struct ZLayout {
  size_t offsets, chunk_off, chunk_series, part, total;
  int64_t chunks;
  bool multi;                   // some series spans several chunks
};

ZLayout znorm_layout(const int32_t* h_lens, int32_t batch) {
  ZLayout L{};
  for (int32_t b = 0; b < batch; ++b) {
    const int64_t c = sdtw::znorm_chunks_of(h_lens[b]);
    L.chunks += c;
    L.multi = L.multi || c > 1;
  }
  size_t at = 0;
  L.offsets = at;
  at = align_up(at + sizeof(int64_t) * ((size_t)batch + 1), kAlign);
  L.chunk_off = at;
  at = align_up(at + sizeof(int64_t) * ((size_t)batch + 1), kAlign);
  L.chunk_series = at;
  at = align_up(at + sizeof(int32_t) * (size_t)L.chunks, kAlign);
  L.part = at;
  at = align_up(at + 2 * sizeof(double) * (size_t)L.chunks, kAlign);
  L.total = at;
  return L;
}

int launch(const void* fn, dim3 grid, dim3 block, void** args, hipStream_t stream) {
  hipError_t e = hipLaunchKernel(fn, grid, block, args, 0, stream);
  return e == hipSuccess ? SDTW_OK : SDTW_ERR_HIP;
}

// Parameters shared by the walk-back entry points (sdtw_backward, sdtw_align).
sdtw::BwdParams bwd_params(const float* queries, const int32_t* query_lens, int32_t batch,
                           const float* reference, int64_t ref_len, const float* cost,
                           const int64_t* end_pos, const float* ckpt, int32_t ckpt_every,
                           int64_t nck, int64_t total, int32_t nmax, const BwdLayout& L,
                           void* workspace) {
  char* ws = static_cast<char*>(workspace);
  int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offsets);
  sdtw::BwdParams p{};
  p.queries = queries;
  p.lens = query_lens;
  p.offsets = offs;
  p.reference = reference;
  p.cost = cost;
  p.end_pos = end_pos;
  p.ckpt = ckpt;
  p.rowck = nck > 0 ? ckpt + total * nck : nullptr;
  p.ref_part = reinterpret_cast<float*>(ws + L.part);
  p.path_lo = reinterpret_cast<int32_t*>(ws + L.lo);
  p.row_lo = reinterpret_cast<int32_t*>(ws + L.row_lo);
  p.row_hi = reinterpret_cast<int32_t*>(ws + L.row_hi);
  p.state = reinterpret_cast<int32_t*>(ws + L.state);
  p.codes = reinterpret_cast<uint32_t*>(ws + L.codes);
  p.part_stride = row_stride_floats(ref_len);
  p.batch = batch;
  p.ref_len = (int32_t)ref_len;
  p.ckpt_every = ckpt_every;
  p.n_ckpt = (int32_t)nck;
  p.nseg = L.nseg;
  p.slots = L.slots;
  p.max_rows = nmax;
  p.round = 0;
  p.nband = 1;
  p.band_rows = sdtw::kRowCkpt;
  p.code_half = L.code_half;
  return p;
}

// The walk itself: offsets, walker state, round 0's recompute, then the
// rounds (walk of round r beside the recompute of round r+1).  Leaves the
// path bounds in p.row_lo, p.row_hi and p.path_lo.
int bwd_walk(sdtw::BwdParams& p, const BwdLayout& L, const int32_t* query_lens, int32_t batch,
             int32_t nmax, bool sq, hipStream_t stream) {
  int64_t* offs = const_cast<int64_t*>(p.offsets);
  int rc;
  {
    int32_t rows = 0;
    int32_t* ranks = nullptr;
    void* args[] = {(void*)&query_lens, (void*)&batch, (void*)&offs, (void*)&rows,
                    (void*)&ranks};
    rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_offsets_kernel), dim3(1),
                dim3(sdtw::kScanThreads), args, stream);
    if (rc != SDTW_OK) return rc;
  }
  {
    void* args[] = {(void*)&p};
    rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_bwd_init_kernel),
                dim3((batch + sdtw::kInitThreads - 1) / sdtw::kInitThreads),
                dim3(sdtw::kInitThreads), args, stream);
    if (rc != SDTW_OK) return rc;
  }
  const size_t round_lds = sdtw::bwd_round_lds_bytes(nmax);      // per wavefront
  const int round_wpg = (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / round_lds));
  // Row bands: later rounds' blocks (few queries still walking, so bound by
  // one block's latency rather than by issue slots) are recomputed as
  // bands from the forward's row checkpoints.
  auto bands = [&](int rows) -> int32_t {
    return p.rowck != nullptr ? (nmax + rows - 1) / rows : 1;
  };
  {
    const void* dirs = sq ? reinterpret_cast<const void*>(&sdtw::sdtw_bwd_dirs_kernel<0>)
                          : reinterpret_cast<const void*>(&sdtw::sdtw_bwd_dirs_kernel<1>);
    p.nband = 1;
    // up to four wavefronts per workgroup, each with its own query and left
    // column in LDS (at most 64 KB per workgroup)
    const size_t per_wave = sizeof(float) * 2 * (size_t)nmax;
    const int wpg = (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / per_wave));
    const int64_t items = (int64_t)batch * L.slots;
    void* args[] = {(void*)&p};
    if (hipLaunchKernel(dirs, dim3((unsigned)((items + wpg - 1) / wpg)), dim3(sdtw::kWave * wpg),
                        args, per_wave * wpg, stream) != hipSuccess)
      return SDTW_ERR_HIP;
  }
  const void* round_fn = sq ? reinterpret_cast<const void*>(&sdtw::sdtw_bwd_round_kernel<0>)
                            : reinterpret_cast<const void*>(&sdtw::sdtw_bwd_round_kernel<1>);
  for (int r = 0; r < L.rounds; ++r) {
    p.round = r;
    // (no next round: no recompute wavefronts, padding ones included)
    p.band_rows = kBandRows;
    p.nband = r + 1 == L.rounds ? 0 : (r >= kFirstBandedKernel ? bands(p.band_rows) : 1);
    const int64_t grid = (int64_t)batch * (1 + (int64_t)L.slots * p.nband);
    void* args[] = {(void*)&p};
    if (hipLaunchKernel(round_fn, dim3((unsigned)((grid + round_wpg - 1) / round_wpg)),
                        dim3(sdtw::kWave * round_wpg), args, round_lds * round_wpg,
                        stream) != hipSuccess)
      return SDTW_ERR_HIP;
  }
  return SDTW_OK;
}

// Binary16 form: queries go in pairs (2i, 2i+1) of equal length, one per
// half of each packed value; returns the pair lengths, or an empty vector if
// a pair's lengths differ.
std::vector<int32_t> f16_pair_lens(const int32_t* h_lens, int32_t batch) {
  std::vector<int32_t> pl((size_t)(batch + 1) / 2);
  for (int32_t i = 0; 2 * i < batch; ++i) {
    if (2 * i + 1 < batch && h_lens[2 * i + 1] != h_lens[2 * i]) return {};
    pl[(size_t)i] = h_lens[2 * i];
  }
  return pl;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

const char* sdtw_status_string(int status) {
  switch (status) {
    case SDTW_OK: return "ok";
    case SDTW_ERR_INVALID_ARG: return "invalid argument";
    case SDTW_ERR_WORKSPACE: return "workspace too small";
    case SDTW_ERR_UNSUPPORTED: return "unsupported variant or shape";
    case SDTW_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int32_t sdtw_variant_count(void) { return variant_count(); }

int sdtw_variant_info(int32_t v, int32_t* rows_per_lane, int32_t* tile_cols, int32_t* waves,
                      int32_t* steps_per_barrier, int32_t* lane_exchange) {
  if (v < 0 || v >= variant_count()) return SDTW_ERR_UNSUPPORTED;
  const Variant& x = variant(v);
  if (rows_per_lane) *rows_per_lane = x.R;
  if (tile_cols) *tile_cols = x.T;
  if (waves) *waves = x.W;
  if (steps_per_barrier) *steps_per_barrier = x.KS;
  if (lane_exchange) *lane_exchange = x.XL;
  return SDTW_OK;
}

int32_t sdtw_default_variant(const int32_t* h_query_lens, int32_t batch, int64_t ref_len,
                             int32_t flags) {
  if (!lens_ok(h_query_lens, batch, nullptr, nullptr) || !ref_ok(ref_len)) return -1;
  return pick_variant(h_query_lens, batch, ref_len, flags, device_cus());
}

size_t sdtw_forward_workspace_bytes(const int32_t* h_query_lens, int32_t batch, int64_t ref_len,
                                    int32_t flags, int32_t variant_id) {
  if (!lens_ok(h_query_lens, batch, nullptr, nullptr) || !ref_ok(ref_len)) return 0;
  if (!fwd_flags_ok(flags)) return 0;
  if (variant_id < -1 || variant_id >= variant_count()) return 0;
  const int cus = device_cus();
  const int vid = variant_id >= 0 ? variant_id
                                  : pick_variant(h_query_lens, batch, ref_len, flags, cus);
  const int64_t slots = fwd_slots(variant(vid), h_query_lens, batch, flags, cus);
  return fwd_layout(batch, ref_len, flags, slots).total;
}

size_t sdtw_checkpoint_floats(const int32_t* h_query_lens, int32_t batch, int64_t ref_len,
                              int32_t ckpt_every) {
  int64_t total = 0;
  if (!lens_ok(h_query_lens, batch, &total, nullptr) || !ref_ok(ref_len) || ckpt_every < 1)
    return 0;
  const int64_t nck = n_ckpt_of(ref_len, ckpt_every);
  return nck > 0 ? (size_t)(total * nck + row_ckpt_rows(total) * ref_len) : 0;
}

}  // extern "C"

namespace {

// sdtw_forward and sdtw_forward_pruned: kind is kSquared, kAbsolute or
// kPruned (threshold tau; no checkpoints).
int forward_impl(const float* queries, const int32_t* h_query_lens, const int32_t* query_lens,
                 int32_t batch, const float* reference, int64_t ref_len, int cost_kind, float tau,
                 float* cost, int64_t* end_pos, float* ckpt, int32_t ckpt_every, int32_t variant_id,
                 int32_t flags, void* workspace, size_t workspace_bytes, void* stream_ptr,
                 bool use_scratch = false) {
  int64_t total = 0;
  int32_t nmax = 0;
  if (!queries || !query_lens || !reference || !cost || !end_pos || (!workspace && !use_scratch))
    return SDTW_ERR_INVALID_ARG;
  if (!lens_ok(h_query_lens, batch, &total, &nmax) || !ref_ok(ref_len))
    return SDTW_ERR_INVALID_ARG;
  if (!fwd_flags_ok(flags)) return SDTW_ERR_INVALID_ARG;
  if (!use_scratch && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return SDTW_ERR_INVALID_ARG;
  const bool want_ckpt = (flags & SDTW_F_CHECKPOINT) != 0;
  int64_t nck = 0;
  if (want_ckpt) {
    if (ckpt_every < 1 || ckpt_every % kCkptQuantum != 0) return SDTW_ERR_INVALID_ARG;
    nck = n_ckpt_of(ref_len, ckpt_every);
    if (nck > 0 && ckpt == nullptr) return SDTW_ERR_INVALID_ARG;
  }
  if (variant_id < -1 || variant_id >= variant_count()) return SDTW_ERR_UNSUPPORTED;
  const bool persistent = (flags & SDTW_F_PERSISTENT) != 0;
  const int cus = device_cus();
  const int vid = variant_id >= 0 ? variant_id
                                  : pick_variant(h_query_lens, batch, ref_len, flags, cus);
  const Variant& v = variant(vid);
  // the uint8-code kernel indexes the row buffer by query
  const int64_t slots = cost_kind == kU8Codes ? batch
                                              : fwd_slots(v, h_query_lens, batch, flags, cus);
  const FwdLayout L = fwd_layout(batch, ref_len, flags, slots);
  if (use_scratch) {
    // the library's own array (256-byte aligned), checked against its size
    // before any HIP call
    if (L.total > SDTW_NOALLOC_SCRATCH_BYTES) return SDTW_ERR_WORKSPACE;
    workspace = scratch_address();
    if (workspace == nullptr) return SDTW_ERR_HIP;
  } else if (workspace_bytes < L.total) {
    return SDTW_ERR_WORKSPACE;
  }
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
  char* ws = static_cast<char*>(workspace);

  FwdParams p{};
  p.queries = queries;
  p.lens = query_lens;
  p.offsets = nullptr;
  p.ranks = nullptr;
  p.reference = reference;
  p.rowbuf = reinterpret_cast<float*>(ws + L.rowbuf);
  p.cost = cost;
  p.end_pos = end_pos;
  p.ckpt = (want_ckpt && nck > 0) ? ckpt : nullptr;
  p.rowck = p.ckpt != nullptr ? ckpt + total * nck : nullptr;
  p.order = reinterpret_cast<int32_t*>(ws + L.order);
  p.queue = reinterpret_cast<int32_t*>(ws + L.queue);
  p.row_stride = row_stride_floats(ref_len);
  p.batch = batch;
  p.ref_len = (int32_t)ref_len;
  p.ckpt_every = want_ckpt ? ckpt_every : 0;
  p.n_ckpt = (int32_t)nck;
  p.prune_tau = tau;
  const int ck = p.ckpt != nullptr ? 1 : 0;
  const bool pruned = cost_kind == sdtw::kPruned;

  if (batch > kInKernelOffsetBatch) {
    // offset and row-buffer slot tables; smaller batches let each workgroup
    // sum the lengths before its query instead
    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offsets);
    int32_t* ranks = reinterpret_cast<int32_t*>(ws + L.ranks);
    int32_t rows = 64 * v.R * v.W;
    void* args[] = {(void*)&query_lens, (void*)&batch, (void*)&offs, (void*)&rows,
                    (void*)&ranks};
    int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_offsets_kernel), dim3(1),
                    dim3(sdtw::kScanThreads), args, stream);
    if (rc != SDTW_OK) return rc;
    p.offsets = offs;
    p.ranks = ranks;
  }
  if (cost_kind == kU8Codes) {
    void* args[] = {(void*)&p};
    return launch(v.u8, dim3(batch), dim3(64 * v.W), args, stream);
  }
  if (persistent) {
    int32_t* order = reinterpret_cast<int32_t*>(ws + L.order);
    int32_t* queue = reinterpret_cast<int32_t*>(ws + L.queue);
    int32_t rows = 64 * v.R * v.W;
    // the smallest last pass the kernel runs, in quarter passes (its tail
    // forms: R/4, R/2 and 3R/4 rows per lane from R = 8, R/2 from R = 4;
    // none with checkpoints)
    int32_t min_quarters = ck ? 4 : (v.R >= 8 ? 1 : (v.R >= 4 ? 2 : 4));
    void* oargs[] = {(void*)&query_lens, (void*)&batch, (void*)&rows, (void*)&min_quarters,
                     (void*)&order, (void*)&queue};
    int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_order_kernel), dim3(1),
                    dim3(sdtw::kScanThreads), oargs, stream);
    if (rc != SDTW_OK) return rc;
    const int grid = (int)persistent_grid_for(v, batch, cus, flags);
    void* args[] = {(void*)&p};
    return launch(pruned ? v.pruned[1] : v.persistent[cost_kind][ck], dim3(grid),
                  dim3(64 * v.W * sdtw::persistent_teams(v.W)), args, stream);
  }
  void* args[] = {(void*)&p};
  return launch(pruned ? v.pruned[0] : v.plain[cost_kind][ck], dim3(batch), dim3(64 * v.W),
                args, stream);
}

}  // namespace

extern "C" {

int sdtw_forward(const float* queries, const int32_t* h_query_lens, const int32_t* query_lens,
                 int32_t batch, const float* reference, int64_t ref_len, int32_t cost_kind,
                 float* cost, int64_t* end_pos, float* ckpt, int32_t ckpt_every, int32_t variant_id,
                 int32_t flags, void* workspace, size_t workspace_bytes, void* stream_ptr) {
  if (cost_kind != SDTW_COST_SQUARED && cost_kind != SDTW_COST_ABSOLUTE)
    return SDTW_ERR_INVALID_ARG;
  return forward_impl(queries, h_query_lens, query_lens, batch, reference, ref_len, cost_kind,
                      0.0f, cost, end_pos, ckpt, ckpt_every, variant_id, flags, workspace,
                      workspace_bytes, stream_ptr);
}

int sdtw_forward_noalloc(const float* queries, const int32_t* h_query_lens,
                         const int32_t* query_lens, int32_t batch, const float* reference,
                         int64_t ref_len, int32_t cost_kind, float* cost, int64_t* end_pos,
                         float* ckpt, int32_t ckpt_every, int32_t variant_id, int32_t flags,
                         void* stream_ptr) {
  if (cost_kind != SDTW_COST_SQUARED && cost_kind != SDTW_COST_ABSOLUTE)
    return SDTW_ERR_INVALID_ARG;
  return forward_impl(queries, h_query_lens, query_lens, batch, reference, ref_len, cost_kind,
                      0.0f, cost, end_pos, ckpt, ckpt_every, variant_id, flags, nullptr, 0,
                      stream_ptr, true);
}

int sdtw_forward_pruned(const float* queries, const int32_t* h_query_lens,
                        const int32_t* query_lens, int32_t batch, const float* reference,
                        int64_t ref_len, float prune_tau, float* cost, int64_t* end_pos,
                        int32_t variant_id, int32_t flags, void* workspace,
                        size_t workspace_bytes, void* stream_ptr) {
  if (prune_tau != prune_tau) return SDTW_ERR_INVALID_ARG;          // NaN
  if (flags & SDTW_F_CHECKPOINT) return SDTW_ERR_INVALID_ARG;       // no checkpoints
  return forward_impl(queries, h_query_lens, query_lens, batch, reference, ref_len,
                      sdtw::kPruned, prune_tau, cost, end_pos, nullptr, 0, variant_id, flags,
                      workspace, workspace_bytes, stream_ptr);
}

size_t sdtw_forward_u8_workspace_bytes(const int32_t* h_query_lens, int32_t batch,
                                       int64_t ref_len) {
  int64_t total = 0;
  if (!lens_ok(h_query_lens, batch, &total, nullptr) || !ref_ok(ref_len)) return 0;
  return u8_layout(batch, total, ref_len).total;
}

int sdtw_forward_u8(const float* queries, const int32_t* h_query_lens, const int32_t* query_lens,
                    int32_t batch, const float* reference, int64_t ref_len, float* cost,
                    int64_t* end_pos, float* codebook, int32_t variant_id, void* workspace,
                    size_t workspace_bytes, void* stream_ptr) {
  int64_t total = 0;
  if (!queries || !query_lens || !reference || !cost || !end_pos || !codebook ||
      !workspace)
    return SDTW_ERR_INVALID_ARG;
  if (!lens_ok(h_query_lens, batch, &total, nullptr) || !ref_ok(ref_len))
    return SDTW_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return SDTW_ERR_INVALID_ARG;
  if (variant_id < -1 || variant_id >= variant_count()) return SDTW_ERR_UNSUPPORTED;
  const U8Layout L = u8_layout(batch, total, ref_len);
  if (workspace_bytes < L.total) return SDTW_ERR_WORKSPACE;
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
  char* ws = static_cast<char*>(workspace);
  uint8_t* qcodes = reinterpret_cast<uint8_t*>(ws + L.qcodes);
  uint8_t* rcodes = reinterpret_cast<uint8_t*>(ws + L.rcodes);
  float2* part = reinterpret_cast<float2*>(ws + L.part);
  sdtw::QBook* book = reinterpret_cast<sdtw::QBook*>(ws + L.book);
  {
    void* args[] = {(void*)&reference, (void*)&ref_len, (void*)&part};
    int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_u8_minmax_kernel), dim3(L.nparts),
                    dim3(sdtw::kQThreads), args, stream);
    if (rc != SDTW_OK) return rc;
  }
  {
    int nparts = L.nparts;
    void* args[] = {(void*)&part, (void*)&nparts, (void*)&book, (void*)&codebook};
    int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_u8_book_kernel), dim3(1),
                    dim3(sdtw::kQThreads), args, stream);
    if (rc != SDTW_OK) return rc;
  }
  const struct { const float* x; int64_t n; uint8_t* c; } enc[2] = {
      {queries, total, qcodes}, {reference, ref_len, rcodes}};
  for (const auto& e : enc) {
    const float* x = e.x;
    int64_t n = e.n;
    uint8_t* c = e.c;
    const int grid = (int)std::min<int64_t>((n + sdtw::kQThreads - 1) / sdtw::kQThreads, 8192);
    void* args[] = {(void*)&x, (void*)&n, (void*)&book, (void*)&c};
    int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_u8_encode_kernel), dim3(grid),
                    dim3(sdtw::kQThreads), args, stream);
    if (rc != SDTW_OK) return rc;
  }
  // The DP itself: the plain forward over the codes (one byte per element).
  return forward_impl(reinterpret_cast<const float*>(qcodes), h_query_lens, query_lens, batch,
                      reinterpret_cast<const float*>(rcodes), ref_len, kU8Codes, 0.0f,
                      cost, end_pos, nullptr, 0, variant_id, 0, workspace, L.fwd.total,
                      stream_ptr);
}

size_t sdtw_forward_f16_workspace_bytes(const int32_t* h_query_lens, int32_t batch,
                                        int64_t ref_len) {
  if (!lens_ok(h_query_lens, batch, nullptr, nullptr) || !ref_ok(ref_len)) return 0;
  if (f16_pair_lens(h_query_lens, batch).empty()) return 0;
  return fwd_layout(batch, ref_len, 0, (batch + 1) / 2).total;
}

int sdtw_forward_f16(const float* queries, const int32_t* h_query_lens,
                     const int32_t* query_lens, int32_t batch, const float* reference,
                     int64_t ref_len, int32_t cost_kind, float* cost, int64_t* end_pos,
                     int32_t variant_id, void* workspace, size_t workspace_bytes,
                     void* stream_ptr) {
  if (!queries || !query_lens || !reference || !cost || !end_pos || !workspace)
    return SDTW_ERR_INVALID_ARG;
  if (!lens_ok(h_query_lens, batch, nullptr, nullptr) || !ref_ok(ref_len))
    return SDTW_ERR_INVALID_ARG;
  if (cost_kind != SDTW_COST_SQUARED && cost_kind != SDTW_COST_ABSOLUTE)
    return SDTW_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return SDTW_ERR_INVALID_ARG;
  const std::vector<int32_t> pl = f16_pair_lens(h_query_lens, batch);
  if (pl.empty()) return SDTW_ERR_UNSUPPORTED;
  if (variant_id < -1 || variant_id >= variant_count()) return SDTW_ERR_UNSUPPORTED;
  const int32_t pairs = (batch + 1) / 2;
  const FwdLayout L = fwd_layout(batch, ref_len, 0, pairs);
  if (workspace_bytes < L.total) return SDTW_ERR_WORKSPACE;
  const int vid = variant_id >= 0 ? variant_id
                                  : pick_variant(pl.data(), pairs, ref_len, 0, device_cus());
  const Variant& v = variant(vid);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
  char* ws = static_cast<char*>(workspace);

  FwdParams p{};
  p.queries = queries;
  p.lens = query_lens;
  p.reference = reference;
  p.rowbuf = reinterpret_cast<float*>(ws + L.rowbuf);
  p.cost = cost;
  p.end_pos = end_pos;
  p.ckpt = nullptr;
  p.row_stride = row_stride_floats(ref_len);
  p.batch = batch;
  p.ref_len = (int32_t)ref_len;
  if (batch > kInKernelOffsetBatch) {
    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offsets);
    int32_t rows = 0;
    int32_t* ranks = nullptr;
    void* args[] = {(void*)&query_lens, (void*)&batch, (void*)&offs, (void*)&rows,
                    (void*)&ranks};
    int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_offsets_kernel), dim3(1),
                    dim3(sdtw::kScanThreads), args, stream);
    if (rc != SDTW_OK) return rc;
    p.offsets = offs;
  } else {
    p.offsets = nullptr;            // each workgroup sums the lengths before its pair
  }
  void* args[] = {(void*)&p};
  return launch(v.half[cost_kind], dim3(pairs), dim3(64 * v.W), args, stream);
}

size_t sdtw_backward_workspace_bytes(const int32_t* h_query_lens, int32_t batch, int64_t ref_len,
                                     int32_t ckpt_every) {
  int64_t total = 0;
  int32_t nmax = 0;
  if (!lens_ok(h_query_lens, batch, &total, &nmax) || !ref_ok(ref_len) || ckpt_every < 1 ||
      ckpt_every % kCkptQuantum != 0)
    return 0;
  if (nmax > sdtw::kDirMaxRows) return 0;
  return bwd_layout(batch, total, ref_len, ckpt_every).total;
}

int sdtw_backward(const float* queries, const int32_t* h_query_lens, const int32_t* query_lens,
                  int32_t batch, const float* reference, int64_t ref_len, int32_t cost_kind,
                  const float* grad_cost, const float* cost, const int64_t* end_pos,
                  const float* ckpt,
                  int32_t ckpt_every, float* grad_queries, float* grad_reference, void* workspace,
                  size_t workspace_bytes, void* stream_ptr) {
  int64_t total = 0;
  int32_t nmax = 0;
  if (!queries || !query_lens || !reference || !grad_cost || !cost || !end_pos ||
      !grad_queries || !grad_reference || !workspace)
    return SDTW_ERR_INVALID_ARG;
  if (!lens_ok(h_query_lens, batch, &total, &nmax) || !ref_ok(ref_len))
    return SDTW_ERR_INVALID_ARG;
  if (cost_kind != SDTW_COST_SQUARED && cost_kind != SDTW_COST_ABSOLUTE)
    return SDTW_ERR_INVALID_ARG;
  if (ckpt_every < 1 || ckpt_every % kCkptQuantum != 0) return SDTW_ERR_INVALID_ARG;
  const int64_t nck = n_ckpt_of(ref_len, ckpt_every);
  if (nck > 0 && ckpt == nullptr) return SDTW_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return SDTW_ERR_INVALID_ARG;
  if (nmax > sdtw::kDirMaxRows) return SDTW_ERR_UNSUPPORTED;
  const BwdLayout L = bwd_layout(batch, total, ref_len, ckpt_every);
  if (workspace_bytes < L.total) return SDTW_ERR_WORKSPACE;

  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
  sdtw::BwdParams p = bwd_params(queries, query_lens, batch, reference, ref_len, cost, end_pos,
                                 ckpt, ckpt_every, nck, total, nmax, L, workspace);
  p.grad_cost = grad_cost;
  p.grad_q = grad_queries;
  const bool sq = cost_kind == SDTW_COST_SQUARED;
  const int rc = bwd_walk(p, L, query_lens, batch, nmax, sq, stream);
  if (rc != SDTW_OK) return rc;
  {
    const bool qlds = sdtw::bwd_grad_q_in_lds(nmax);
    const void* grad =
        sq ? (qlds ? reinterpret_cast<const void*>(&sdtw::sdtw_bwd_grad_kernel<0, true>)
                   : reinterpret_cast<const void*>(&sdtw::sdtw_bwd_grad_kernel<0, false>))
           : (qlds ? reinterpret_cast<const void*>(&sdtw::sdtw_bwd_grad_kernel<1, true>)
                   : reinterpret_cast<const void*>(&sdtw::sdtw_bwd_grad_kernel<1, false>));
    void* args[] = {(void*)&p};
    const dim3 grid(batch, sdtw::kGradColGroups + sdtw::bwd_grad_row_groups(nmax));
    if (hipLaunchKernel(grad, grid, dim3(sdtw::kGradThreads), args,
                        sdtw::bwd_grad_lds_bytes(nmax), stream) != hipSuccess)
      return SDTW_ERR_HIP;
  }
  {
    const float* part = p.ref_part;
    int64_t stride = p.part_stride;
    const int32_t* lo = p.path_lo;
    int32_t m = p.ref_len;
    void* args[] = {(void*)&part, (void*)&stride, (void*)&lo, (void*)&end_pos, (void*)&batch,
                    (void*)&m, (void*)&grad_reference};
    const int grid = (int)((ref_len + sdtw::kRefReduceThreads - 1) / sdtw::kRefReduceThreads);
    return launch(reinterpret_cast<const void*>(&sdtw::sdtw_ref_reduce_kernel), dim3(grid),
                  dim3(sdtw::kRefReduceThreads), args, stream);
  }
}

size_t sdtw_align_workspace_bytes(const int32_t* h_query_lens, int32_t batch, int64_t ref_len,
                                  int32_t ckpt_every) {
  int64_t total = 0;
  int32_t nmax = 0;
  if (!lens_ok(h_query_lens, batch, &total, &nmax) || !ref_ok(ref_len) || ckpt_every < 1 ||
      ckpt_every % kCkptQuantum != 0)
    return 0;
  if (nmax > sdtw::kDirMaxRows) return 0;
  return bwd_layout(batch, total, ref_len, ckpt_every, false).total;
}

int sdtw_align(const float* queries, const int32_t* h_query_lens, const int32_t* query_lens,
               int32_t batch, const float* reference, int64_t ref_len, int32_t cost_kind,
               const float* cost, const int64_t* end_pos, const float* ckpt, int32_t ckpt_every,
               int64_t* start_pos, int32_t* path_lo, int32_t* path_hi, void* workspace,
               size_t workspace_bytes, void* stream_ptr) {
  int64_t total = 0;
  int32_t nmax = 0;
  if (!queries || !query_lens || !reference || !cost || !end_pos || !start_pos || !path_lo ||
      !path_hi || !workspace)
    return SDTW_ERR_INVALID_ARG;
  if (!lens_ok(h_query_lens, batch, &total, &nmax) || !ref_ok(ref_len))
    return SDTW_ERR_INVALID_ARG;
  if (cost_kind != SDTW_COST_SQUARED && cost_kind != SDTW_COST_ABSOLUTE)
    return SDTW_ERR_INVALID_ARG;
  if (ckpt_every < 1 || ckpt_every % kCkptQuantum != 0) return SDTW_ERR_INVALID_ARG;
  const int64_t nck = n_ckpt_of(ref_len, ckpt_every);
  if (nck > 0 && ckpt == nullptr) return SDTW_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return SDTW_ERR_INVALID_ARG;
  if (nmax > sdtw::kDirMaxRows) return SDTW_ERR_UNSUPPORTED;
  const BwdLayout L = bwd_layout(batch, total, ref_len, ckpt_every, false);
  if (workspace_bytes < L.total) return SDTW_ERR_WORKSPACE;

  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
  sdtw::BwdParams p = bwd_params(queries, query_lens, batch, reference, ref_len, cost, end_pos,
                                 ckpt, ckpt_every, nck, total, nmax, L, workspace);
  p.ref_part = nullptr;
  p.row_lo = path_lo;                           // the walker writes the bounds in place
  p.row_hi = path_hi;
  const int rc = bwd_walk(p, L, query_lens, batch, nmax, cost_kind == SDTW_COST_SQUARED, stream);
  if (rc != SDTW_OK) return rc;
  const int32_t* lo = p.path_lo;
  void* args[] = {(void*)&lo, (void*)&batch, (void*)&start_pos};
  return launch(reinterpret_cast<const void*>(&sdtw::sdtw_align_start_kernel),
                dim3((batch + sdtw::kInitThreads - 1) / sdtw::kInitThreads),
                dim3(sdtw::kInitThreads), args, stream);
}

size_t sdtw_workspace_bytes(const int32_t* h_query_lens, int32_t batch, int64_t ref_len,
                            int32_t flags, int32_t ckpt_every) {
  const size_t fwd = sdtw_forward_workspace_bytes(h_query_lens, batch, ref_len, flags, -1);
  if (fwd == 0 || !(flags & SDTW_F_CHECKPOINT)) return fwd;
  const size_t bwd = sdtw_backward_workspace_bytes(h_query_lens, batch, ref_len, ckpt_every);
  const size_t aln = sdtw_align_workspace_bytes(h_query_lens, batch, ref_len, ckpt_every);
  if (bwd == 0 || aln == 0) return 0;
  return std::max({fwd, bwd, aln});
}

size_t sdtw_znorm_workspace_bytes(const int32_t* h_lens, int32_t batch) {
  if (!lens_ok(h_lens, batch, nullptr, nullptr)) return 0;
  return znorm_layout(h_lens, batch).total;
}

int sdtw_znorm(const float* x, const int32_t* h_lens, const int32_t* lens, int32_t batch,
               float* z, void* workspace, size_t workspace_bytes, void* stream_ptr) {
  if (!x || !lens || !z || !workspace) return SDTW_ERR_INVALID_ARG;
  if (!lens_ok(h_lens, batch, nullptr, nullptr)) return SDTW_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return SDTW_ERR_INVALID_ARG;
  const ZLayout L = znorm_layout(h_lens, batch);
  if (workspace_bytes < L.total) return SDTW_ERR_WORKSPACE;
  if (L.chunks > INT32_MAX) return SDTW_ERR_UNSUPPORTED;
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
  char* ws = static_cast<char*>(workspace);
  if (batch <= sdtw::kZDirectBatch) {
    // direct form: the host lists the long series and every stride-th
    // series' first element (it knows both from the host lengths)
    sdtw::ZDirect d{};
    d.stride = (batch + sdtw::kZCoarse - 1) / sdtw::kZCoarse;
    int64_t off = 0;
    int32_t long_chunks = 0;
    bool fits = true;
    for (int32_t b = 0; b < batch && fits; ++b) {
      if (b % d.stride == 0) d.prefix[b / d.stride] = off;
      if (h_lens[b] > sdtw::kZWaveMax) {
        if (d.nlong == sdtw::kZMaxLong) {
          fits = false;
          break;
        }
        const int32_t nch = (int32_t)sdtw::znorm_chunks_of(h_lens[b]);
        d.lg[d.nlong] = sdtw::ZLong{off, b, h_lens[b], long_chunks, nch};
        ++d.nlong;
        long_chunks += nch;
      }
      off += h_lens[b];
    }
    if (fits) {
      d.x = x;
      d.z = z;
      d.lens = lens;
      d.part = reinterpret_cast<double*>(ws + L.part);
      d.batch = batch;
      d.long_chunks = long_chunks;
      void* args[] = {(void*)&d};
      constexpr int wpg = sdtw::kZWavesPerWG;
      int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_znorm_direct_kernel),
                      dim3((unsigned)((batch + long_chunks + wpg - 1) / wpg)),
                      dim3(sdtw::kZThreads), args, stream);
      if (rc != SDTW_OK || long_chunks == 0) return rc;
      return launch(reinterpret_cast<const void*>(&sdtw::sdtw_znorm_long_apply_kernel),
                    dim3((unsigned)((long_chunks + wpg - 1) / wpg)), dim3(sdtw::kZThreads),
                    args, stream);
    }
  }
  // table form
  sdtw::ZParams p{};
  p.x = x;
  p.z = z;
  p.lens = lens;
  p.offsets = reinterpret_cast<int64_t*>(ws + L.offsets);
  p.chunk_off = reinterpret_cast<int64_t*>(ws + L.chunk_off);
  p.chunk_series = reinterpret_cast<int32_t*>(ws + L.chunk_series);
  p.part = reinterpret_cast<double*>(ws + L.part);
  p.batch = batch;
  {
    int64_t* off = reinterpret_cast<int64_t*>(ws + L.offsets);
    int64_t* coff = reinterpret_cast<int64_t*>(ws + L.chunk_off);
    int32_t* cser = reinterpret_cast<int32_t*>(ws + L.chunk_series);
    void* args[] = {(void*)&lens, (void*)&batch, (void*)&off, (void*)&coff, (void*)&cser};
    const int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_znorm_index_kernel), dim3(1),
                          dim3(sdtw::kScanThreads), args, stream);
    if (rc != SDTW_OK) return rc;
  }
  void* args[] = {(void*)&p};
  const dim3 grid((unsigned)L.chunks);
  int rc = launch(reinterpret_cast<const void*>(&sdtw::sdtw_znorm_stats_kernel), grid,
                  dim3(sdtw::kZThreads), args, stream);
  if (rc != SDTW_OK || !L.multi) return rc;
  return launch(reinterpret_cast<const void*>(&sdtw::sdtw_znorm_apply_kernel), grid,
                dim3(sdtw::kZThreads), args, stream);
}

}  // extern "C"
