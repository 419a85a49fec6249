// Host-side structures of the library: the context, workspace arenas and the
// drivers shared by the single-field, batched and serving entry points.
#pragma once

#include <string>
#include <vector>

#include "../../include/exactz.h"
#include "exz_internal.h"

namespace exz {

// Device bytes a context may hold (arenas of the context and of its jobs);
// limit 0 = no limit.
struct Budget {
  size_t limit = 0;
  size_t used = 0;
};

// Freed job arenas kept for later jobs: taking one needs no allocation and,
// unlike hipFree, no wait for the device.  Pooled bytes stay charged to the
// budget (the context still holds them) until they are freed: past the cap
// (largest first), or all at once by trim(), which an allocation that fails
// calls before it gives up.
struct Pool {
  struct Block {
    char *p;
    size_t bytes;
  };
  std::vector<Block> blocks;
  size_t bytes = 0;
  size_t cap = (size_t)32 << 30;  // most bytes kept
  Budget *budget = nullptr;
  // the smallest block of need .. need + need / 4 + 1 MiB bytes, or nullptr
  char *take(size_t need, size_t &got);
  void give(char *p, size_t n);
  void trim();
};

// Growable device buffer carved into 256-byte aligned pieces per call.  A
// fixed arena uses memory it does not own (the no-allocation entry point's
// static buffer): it never allocates or frees, and a reserve beyond its
// capacity fails with hipErrorOutOfMemory.  A fixed arena chained after
// another one starts, at each reserve, where that one's carving ends.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  bool fixed = false;
  char *end = nullptr;          // fixed: end of the usable memory
  const Arena *after = nullptr; // fixed: start after this arena's carving
  Budget *budget = nullptr;     // charged for what this arena allocates
  bool exact = false;           // allocate exactly what is asked (no growth slack)
  Pool *pool = nullptr;         // released memory goes here, and reserve looks here first
  hipError_t reserve(size_t bytes);  // resets the carve offset
  void *take(size_t bytes);
  void release();
  void wrap(void *p, size_t bytes) {
    base = (char *)p;
    end = base + bytes;
    cap = bytes;
    off = 0;
    fixed = true;
    after = nullptr;
  }
  void chain(const Arena *prev, char *limit) {
    base = nullptr;
    end = limit;
    cap = off = 0;
    fixed = true;
    after = prev;
  }
};

// One tile of a radix sort over the critical points of several fields at
// once: the fields' keys lie one after another, every tile within one field,
// and each field's digit histograms form one block (digit-major over the
// field's tiles) after those of the fields before it, so one exclusive scan
// of the concatenated histograms gives every (field, digit, tile) its output
// position: the sum over the earlier fields is where the field's keys start.
struct SortTile {
  uint32_t start;   // first key of the tile
  uint32_t count;   // keys in the tile (<= 4096)
  uint32_t hbase;   // first histogram entry of the tile's field
  uint32_t ntiles;  // tiles of the field
  uint32_t t;       // the tile's index within its field
};
hipError_t launch_radix_sort_tiles(int key_bytes, void *keys, uint32_t *vals, void *keys_tmp,
                                   uint32_t *vals_tmp, uint32_t count, const SortTile *tiles,
                                   uint32_t ntiles, uint32_t *hist, uint32_t *scan_tmp,
                                   size_t scan_words, hipStream_t s);
constexpr uint32_t SORT_TILE = 4096;  // keys per sort tile

// Size accounting that mirrors Arena::take.
struct Layout {
  size_t total = 0;
  size_t add(size_t bytes);
};

exz_status prepare_field(exz_ctx *ctx, const exz_params *p, FieldDev &fd);
exz_status setup_field(exz_ctx *ctx, FieldDev &fd, const void *f, const void *g_hat, void *g_out,
                       uint8_t *cnt_io, int64_t max_iters, Arena &A, Arena &B, hipStream_t s);
// The two halves of setup_field.  Phase A (per-vertex work: validation,
// reference topology, critical-point bitmask and counts) is issued on s and
// ends with copies of the device state into *h_state and of the number of
// critical points into *h_k (both pinned); phase B (the critical points in
// f's order) needs that number.
exz_status setup_phase_a(exz_ctx *ctx, FieldDev &fd, const void *f, const void *g_hat,
                         void *g_out, uint8_t *cnt_io, int64_t max_iters, Arena &A, hipStream_t s,
                         State *h_state, uint32_t *h_k);
exz_status setup_phase_b(exz_ctx *ctx, FieldDev &fd, uint32_t K, Arena &B, hipStream_t s);
exz_status exz_correct_impl(exz_ctx *ctx, const void *f, const void *g_hat, void *g_out,
                            uint8_t *cnt_io, const exz_params *params, exz_result *res,
                            hipStream_t s, Arena &A, Arena &B, Arena &C, bool profile);
// Device address of exz_correct_noalloc's static buffer on `device` (which
// the caller has made current), looked up once per device; its size.
hipError_t scratch_lookup(int device, void **ptr, size_t *bytes);
// f and g 16-byte aligned and the counts 4-byte aligned (apply may then
// read a quad of vertices with vector loads).
inline int quad_aligned(const FieldDev &fd) {
  return ((uintptr_t)fd.f % 16 == 0) && ((uintptr_t)fd.g % 16 == 0) && ((uintptr_t)fd.cnt % 4 == 0);
}

// Bytes of the target marks: one per vertex, then zero padding (apply reads
// marks four at a time), rounded to 16.
inline size_t mark_pad_bytes(const exz::FieldDev &fd) { return ((size_t)fd.n + 64 + 15) / 16 * 16; }
// The marks (zero padded) and the tags of their 256-vertex chunks.
inline size_t mark_bytes(const exz::FieldDev &fd) {
  return mark_pad_bytes(fd) + ((size_t)fd.n + 255) / 256;
}

// Bytes of the dirty-box flags: one per box of the smallest shape.
inline size_t box_flag_count(const exz::FieldDev &fd) {
  return (size_t)fd.tiles_x * (size_t)fd.ny * (size_t)fd.nz;
}
// The flags (padded to 16 bytes) followed by the box list.
inline size_t box_flag_bytes(const exz::FieldDev &fd) {
  return (box_flag_count(fd) + 15) / 16 * 16 + 4 * box_flag_count(fd);
}
inline uint32_t *box_list_of(const exz::FieldDev &fd, char *flags) {
  return (uint32_t *)(flags + (box_flag_count(fd) + 15) / 16 * 16);
}

void layout_a(const FieldDev &fd, bool own_cnt, int trace_cap, bool need_lab, Layout &L,
              size_t off[9]);
void layout_b(const FieldDev &fd, uint32_t K, Layout &L, size_t off[12]);
// 32-bit words of the pointer-jumping convergence bitmask of count labels.
size_t jump_conv_words(uint64_t count);
void layout_c(const FieldDev &fd, bool original, bool certify, Layout &L, size_t off[6]);
exz_status setup_paths(exz_ctx *ctx, FieldDev &fd, bool original, bool certify, Arena &C,
                       uint32_t **lab_g, hipStream_t s);
hipError_t ensure_work_stream(exz_ctx *ctx);

}  // namespace exz

struct exz_ctx {
  int device = 0;
  bool busy = false;
  bool profile = false;
  bool graph = true;
  int poll = 0;     // 0 = adaptive
  int tile_y = 0;  // 0: box shape chosen by the field's dimensionality
  int tile_z = 0;
  int grid_blocks = -1;
  bool frontier = true;
  std::string last_error;
  exz::Budget budget;               // device bytes of the context and its jobs
  exz::Arena H;                     // device copies for exz_correct_host
  void *scratch = nullptr;          // exz_correct_noalloc's buffer on this device
  size_t scratch_bytes = 0;
  uint8_t *d_comp = nullptr;        // link component table (2^14 bytes)
  uint32_t *d_conn = nullptr;       // one-component bits (2^14 bits)
  exz::State *h_state = nullptr;    // pinned
  uint32_t *h_k = nullptr;          // pinned
  exz::Arena A, B, C;
  exz::Arena BA, BB, BC;  // batched correction workspaces (per-vertex, per-CP, paths)
  void *step_host = nullptr;  // exz_step staging: pinned FieldDev array + item lists
  void *step_dev = nullptr;
  size_t step_cap = 0;
  hipEvent_t step_copied = nullptr;  // the host staging of the last step was copied
  hipEvent_t step_done = nullptr;    // the last step's launches (they read step_dev)
  // batched / job launch geometry (0 = default): boxes for 3D and 2D members
  // (tile_y * 100 + tile_z), grid caps of the check and apply passes, and
  // apply item size in quads per thread
  int btile3 = 0, btile2 = 0, bgrid_box = 0, bgrid_apply = 0, bitem = 0;
  hipStream_t work = nullptr;       // internal stream for captured work (default priority)
  // streams (default priority) over which the batched set-up of independent
  // fields is spread, and the events that fork them from / join them to the
  // caller's stream
  static constexpr int NSIDE = 4;
  hipStream_t side[NSIDE] = {};
  hipEvent_t side_ev[NSIDE + 1] = {};
  hipEvent_t order_in = nullptr, order_out = nullptr;
  std::vector<hipEvent_t> events;
  hipEvent_t ev_start = nullptr, ev_setup = nullptr, ev_end = nullptr;
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  // released jobs whose device work had not ended yet; freed once it has
  std::vector<exz_job *> graveyard;
  exz::Pool job_pool;  // the freed arenas of jobs, for later jobs
  // the pinned state blocks and events of freed jobs, for later jobs (freeing
  // pinned memory waits for the device; these are reused instead)
  std::vector<void *> spare_pinned;
  std::vector<hipEvent_t> spare_events;
  static constexpr size_t SPARE_JOBS = 256;
};

// Frees every job of ctx's graveyard (the device must be idle).
void free_graveyard(exz_ctx *ctx);

// A serving job: one field whose correction state stays on the device
// between exz_step calls.
struct exz_job {
  exz_ctx *ctx = nullptr;
  exz::Arena A, B;        // the job's own workspace
  exz::FieldDev fd;
  exz_params params;
  hipStream_t last = nullptr;   // stream of the last work issued for it
  exz_result result;
  bool finished = false;
  hipEvent_t ready = nullptr;  // set-up done (recorded on the creation stream)
  bool joined = false;         // a step has waited for `ready`
  // exz_job_submit: phase A of the set-up is in flight until a_done; phase
  // B is issued on create_stream by the first exz_step / exz_job_query /
  // exz_job_poll that finds it ended
  int phase = 1;               // 0 phase A in flight, 1 set up, 2 failed
  exz_status failed = EXZ_OK;  // phase 2: the status, and its message
  std::string failed_msg;
  hipEvent_t a_done = nullptr;
  hipStream_t create_stream = nullptr;
  // The state after each step goes to one of NSTATE host slots in turn.
  // exz_step lets the host run one step ahead (it waits until the previous
  // step has started), so of the steps issued, the latest two may still run
  // and the third latest has ended: three slots always hold an ended one.
  static constexpr int NSTATE = 3;
  struct Pinned {
    exz::State st[NSTATE];      // phase A's state (slot 0), then the state after each step
    uint32_t k;                // number of critical points
  };
  Pinned *pinned = nullptr;    // host-pinned
  hipEvent_t polled[NSTATE] = {};  // after the copy into st[s] of its last steps
  bool recorded[NSTATE] = {};
  int slot = -1;               // slot of the latest step's copy (-1: not stepped yet)
};
