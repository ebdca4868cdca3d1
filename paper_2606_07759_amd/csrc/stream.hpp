// Streaming kernel of the fused IM build and its kernel-variant record
// (internal header, not part of the ABI).  The variant table is split over
// several translation units so that their instantiations compile in parallel;
// every instantiation lives in exactly one of them.
#pragma once

#include <climits>
#include <utility>

#include "common.hpp"

namespace synim {

constexpr int MAX_TILE_ROWS = 512;   // IF rows one tile may stage

// ------------------------------------------------------------------ streaming

__device__ __forceinline__ float dpp_sum(float v, int lps) {
  // quad_perm [1,0,3,2] then [2,3,0,1]; for 8 lanes also row_half_mirror
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  if (lps == 8)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
  return v;
}

// One (WFS, DM) pair's planned build: its IF stack, its output and its plan.
struct PairDesc {
  const float* ifs;          // [n_act][H_in][W_in]
  float* out;                // plane (out_plane0) of [plane][n_act][2nv]
  const int2* origin;
  const int2* hrows;         // patch rows holding a non-zero weight
  const float* weights;      // plane 0 base
  const int* slot_kk;
  const int4* tile_info;
  const int2* rows;
  int n_act, H_in, W_in, nv;
  int n_tiles, ns, BHmax, chunk;
  int n_chunks, pad0, pad1, pad2;
};

// A batched launch walks "super-chunks": one actuator chunk of one DM, with
// the tiles of every pair that sees that DM.  Super-chunks go round-robin to
// the XCD queues, DM-major, so the pairs sharing a DM read each IF chunk at
// about the same time on one XCD (the IF bytes come from HBM once).
struct SuperChunk {
  int item0;                 // first item of this record in its XCD's queue
  int dm;                    // DM group
  int chunk;                 // actuator chunk of that DM
  int items;                 // sum of the tiles of the group's pairs
};

struct StreamArgs {
  PairDesc one;              // single-pair launches
  const PairDesc* pairs;     // batched launches: pair table (nullptr: single pair)
  const SuperChunk* recs;    // batched: per-XCD records, XCD x at recs[rec_off[x]..]
  const int2* groups;        // batched: per DM (first pair, number of pairs)
  int rec_off[8], rec_cnt[8], xcd_items[8];
  int* counters;             // [gridDim.z][8] work counters, zero at the launch
  float* scratch;            // 64 floats that absorb the stores of idle lanes
  int plane0;                // first weight plane handled (blockIdx.z adds to it)
  int out_plane0;            // weight plane that lands in out[0]
  const float* grad;         // VJP: [n_act][2nv]
  double* partials;          // VJP: [4][gridDim.x]
  // Bounded-lag sync of the workgroups of one XCD (single pair, one chunk
  // per XCD): every sync_every actuators a workgroup waits until each tile of
  // its XCD has started the previous block, so the tiles of a chunk read the
  // rows they share within a few actuators of each other.  0 = off.
  int sync_every;
  int* sync_ctr;             // [gridDim.z][8] block entries, zero at the launch
  const int* n_active;       // non-empty tiles (written by the plan)
  // Batched launches with shared tiles (nullptr jslots: per-pair tiles).  A
  // shared tile gathers the subapertures of every pair of one DM group whose
  // patches fall in one region of the IF grid, so that region is staged once
  // for all of them.
  const int* jslots;         // [tile][jNS]: (pair << 20) | subaperture, or -1; pair
                             // indexes the pair table
  const int4* jinfo;         // [tile] (y0, rows, first column, pitch), written by the plan
  const int2* jrows;         // [tile][jBHmax] (first column, packed offset)
  const int2* jgroups;       // per DM group: (first shared tile, count)
  int jNS, jBHmax;
  // Single-pair launches: the last workgroup to finish sets the n_counters
  // ints from `counters` (work and sync counters) and *finish back to zero,
  // so the next launch on the same plan needs no clearing launch before it.
  // nullptr: the caller clears the counters (batched launches).
  int* finish;
  int n_counters;
};

typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt immediates (gfx9 encoding) that wait on vmcnt only.
constexpr int waitcnt_vm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | (((n >> 4) & 3) << 14); }

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) float gfloat_t;   // global memory

// Raw buffer resource (stride 0, range-checked) over [base, base + bytes),
// every word wave-uniform so it lives in SGPRs.
__device__ __forceinline__ u32x4 buffer_rsrc(const void* base, unsigned bytes) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(base);
  u32x4 r;
  r.x = __builtin_amdgcn_readfirstlane((unsigned)a);
  r.y = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));   // stride 0
  r.z = __builtin_amdgcn_readfirstlane(bytes);
  r.w = 0x00020000u;
  return r;
}

// LDS byte address of a __shared__ location, wave-uniform (M0 operand).
__device__ __forceinline__ unsigned lds_addr(const void* p) {
  return __builtin_amdgcn_readfirstlane(
      (unsigned)(size_t)(lds_void_t*)const_cast<void*>(p));
}

// Compiler-only ordering point: no memory access moves across it.
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Streams one group of actuators' packed tile rows into an LDS stage buffer
// with buffer->LDS DMA.  Each wave issues exactly NJ instructions per stage,
// so the number of vector-memory operations in flight is known at compile
// time.  The buffer resource covers the group's IF planes only: rows
// above/below the grid fall outside its range and read as zero; columns
// outside the grid are sent out of range explicitly.
//
// The DMA is written as inline assembly on purpose: the compiler then tracks
// no LDS write for it and adds no wait of its own before the stage reads
// (its conservative merge at the pipeline loop head drained every DMA in
// flight there).  Completion is the pipeline's explicit vmcnt waits alone.
//
// Two hazards of gfx9 sit between a DMA and the scalar registers it reads,
// and the compiler pads neither around inline assembly (it does around its own
// buffer loads):
//  * a vector-memory instruction that reads an SGPR written by a VALU
//    instruction (here the v_readfirstlane that builds the buffer resource)
//    needs 5 wait states in between, or it may read the SGPR's previous value:
//    the DMA then streams from a stale base address (another actuator's plane,
//    or no valid address at all) or with a stale record count;
//  * an LDS DMA reads M0 (its LDS destination) one cycle after issue, so a
//    scalar write of M0 right before it needs one wait state.
// Each DMA below therefore opens with s_nop 4 (5 wait states), which covers
// both whatever the compiler schedules right before the asm block.
template <int BLOCK, int NJ, int VW>
__device__ __forceinline__ void stage_issue(const float* plane_ptr, int plane_bytes,
                                            const unsigned* voff, float4* buf, int wave) {
  const u32x4 r = buffer_rsrc(plane_ptr, (unsigned)plane_bytes);
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const unsigned m0 =
        lds_addr(reinterpret_cast<float*>(buf) + (size_t)(BLOCK * j + 64 * wave) * VW);
    if constexpr (VW == 4)
      asm volatile("s_nop 4\n\tbuffer_load_dwordx4 %0, %1, 0 offen lds" ::"v"(voff[j]), "s"(r),
                   "{m0}"(m0)
                   : "memory");
    else
      asm volatile("s_nop 4\n\tbuffer_load_dword %0, %1, 0 offen lds" ::"v"(voff[j]), "s"(r),
                   "{m0}"(m0)
                   : "memory");
  }
}

// Stage buffer K of a pipeline: one distinct __shared__ object per K, so the
// compiler can tell that reading one stage never aliases the DMA in flight
// into another (with one shared array it would drain every DMA before each
// LDS read).
template <int K, int F4>
__device__ __forceinline__ float4* stage_buf() {
  __shared__ float4 b[F4];
  return b;
}

// s_waitcnt vmcnt(n) for a wave-uniform runtime n in [0, 63] (the immediate
// must be a constant: a branch over every value).  n is moved to a scalar
// register first: where the compiler cannot prove it uniform it would branch
// on a vector compare per value, with exec-mask bookkeeping at every level.
__device__ __forceinline__ void wait_vm(int n) {
  n = __builtin_amdgcn_readfirstlane(n);
  switch (n) {
#define SYNIM_W(k) case k: __builtin_amdgcn_s_waitcnt(waitcnt_vm(k)); break;
#define SYNIM_W8(k) SYNIM_W(k) SYNIM_W(k + 1) SYNIM_W(k + 2) SYNIM_W(k + 3) SYNIM_W(k + 4) \
    SYNIM_W(k + 5) SYNIM_W(k + 6) SYNIM_W(k + 7)
    SYNIM_W8(0) SYNIM_W8(8) SYNIM_W8(16) SYNIM_W8(24) SYNIM_W8(32) SYNIM_W8(40) SYNIM_W8(48)
    SYNIM_W8(56)
#undef SYNIM_W8
#undef SYNIM_W
    default: __builtin_amdgcn_s_waitcnt(waitcnt_vm(0)); break;
  }
  compiler_fence();
}

// s_barrier with compiler ordering points on both sides: the stage reads of
// the step before stay above it, the reads of the next stage below it.
__device__ __forceinline__ void stage_barrier() {
  compiler_fence();
  __builtin_amdgcn_s_barrier();
  compiler_fence();
}

// XCD sync bookkeeping.  The block-entry counter of a workgroup's XCD is read
// in two ways:
//  * a snapshot that rides with every stage: a 4-byte buffer->LDS DMA of the
//    counter issued just before the stage's IF rows, so the wait that makes
//    the stage visible also makes the snapshot visible, at no extra stall;
//    the load has device scope (sc1, as an agent-scope atomic load), so it
//    sees the other workgroups' atomics;
//  * a device-scope atomic load, only when a snapshot says the peers are
//    behind (the wave then waits for it, draining its own DMA queue).
constexpr int SYNC_SPIN_MAX = 1000;   // polls before a workgroup stops syncing
constexpr int SYNC_STRIDE = 32;       // ints between the counters (own 128-byte line)

__device__ __forceinline__ void snapshot_issue(const int* ctr, int* lds_dst) {
  const u32x4 r = buffer_rsrc(ctr, 4u);
  const unsigned m0 = lds_addr(lds_dst);
  asm volatile("s_nop 4\n\tbuffer_load_dword %0, %1, 0 offen sc1 lds" ::"v"(0u), "s"(r),
               "{m0}"(m0)
               : "memory");
}

// Actuators one stage may hold: PACK (1 = one actuator per stage), cut to
// what keeps every wait count of the pipeline (the later stages' DMA, the
// stores of the steps since, the sync extras) within the vmcnt range.
constexpr int stage_pack(int nj, int nst, int pack) {
  const int vm = (63 - (nst - 2) * (nj + 1) - 1) / (nst - 1);
  return pack <= 1 || vm < 1 ? 1 : (vm < pack ? vm : pack);
}

// Persistent streaming kernel.  Work items are (actuator chunk, tile) pairs;
// workgroup b serves the queue of its XCD (b mod 8 - consecutive workgroups are
// dispatched round-robin over the 8 XCDs), and each queue walks its chunks in
// order, tiles fastest, so the tiles of one chunk run side by side on one XCD
// and share the IF rows of their halos in that XCD's L2.  Within an item the
// actuators stream through NST LDS stages with NST-1 actuators in flight.
// Waves per SIMD the stream kernel runs at when LDS is what limits its
// workgroups per CU (160 KB per CU, at most 8 waves per SIMD): the register
// budget of the 16-byte DMA variants is set to match, so registers never cut
// that occupancy further.  (The 4-byte DMA variants hold four times the DMA
// offsets and keep the compiler's own budget.)
constexpr int stream_waves_per_simd(int block, int nj, int vw, int nst) {
  const int lds = nst * nj * block * vw * 4 + MAX_TILE_ROWS * 8 + 1024;
  int wgs = 160 * 1024 / lds;
  if (wgs * block > 2048) wgs = 2048 / block;
  const int w = wgs * (block / 64) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// BATCH = false: the single-pair launches, with every batch path compiled out.
// BATCH = true: the batched launches; that instantiation keeps the single-pair
// paths too and picks by g.pairs at run time.  (A form with the batch decision
// fixed at compile time once gave wrong values for some actuators from run to
// run.  Its DMA read buffer-resource SGPRs that a v_readfirstlane had written
// one wait state earlier, where 5 are needed; the DMA padding above removes
// that hazard from every form.)
template <int BLOCK, int LPS, int RPL, int PW, int NJ, int VW, int NST, int PACK, bool VJP,
          bool BATCH>
__global__ __launch_bounds__(BLOCK, VW == 4 ? stream_waves_per_simd(BLOCK, NJ, VW, NST) : 1) void
im_stream_kernel(StreamArgs g) {
  constexpr int PH = LPS * RPL;
  constexpr int E = PH * PW;
  constexpr int STAGE_F4 = NJ * BLOCK * VW / 4;   // float4 per stage buffer
  constexpr int KPMAX = stage_pack(NJ, NST, PACK);
  static_assert(NST >= 2 && NST <= 8, "2..8 stages");
  static_assert(NJ * (NST - 2) <= 63, "vmcnt range");
  __shared__ int s_item;
  __shared__ double s_red[BLOCK / 64];
  __shared__ int s_snap[NST];   // per stage: block-entry counter when it was issued
  __shared__ int2 s_rows[MAX_TILE_ROWS];   // the current tile's row table

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int slot = tid / LPS, q = tid % LPS;
  const int xcd = blockIdx.x & 7;
  const int plane = g.plane0 + blockIdx.z;
  // Items of XCD queue x.  A workgroup starts on its own XCD's queue and,
  // once that is empty, takes what is left in the other queues (in order
  // x+1, x+2, ...), so no XCD idles while another still has items.  With
  // the bounded-lag sync on, the workgroups of an XCD must stay on its queue.
  auto queue_items = [&](int x) {
    if (BATCH && g.pairs != nullptr) {
      return g.xcd_items[x];
    } else {
      const int nc_x = g.one.n_chunks > x ? (g.one.n_chunks - x + 7) / 8 : 0;
      return nc_x * g.one.n_tiles;
    }
  };
  const bool may_steal = !((!BATCH || g.pairs == nullptr) && g.sync_every > 0);
  int qx = xcd;
  int n_items = queue_items(qx);
  int* ctr = g.counters + 8 * blockIdx.z + qx;
  // queues other than its own that still held items when the workgroup last
  // looked (bit i: queue xcd + 1 + i); -1 before the first look
  int others = -1;
  __shared__ int s_others;
  double vacc = 0.0;
  // read once, before any DMA: a compiler-tracked load still pending at the
  // pipeline loop head would make the compiler drain the DMA queue there
  const int n_part = (!BATCH || g.pairs == nullptr) && g.sync_every > 0 ? *g.n_active : 0;

  for (;;) {
    __syncthreads();   // the previous item's stage buffers and row table are free again
    if (tid == 0) s_item = atomicAdd(ctr, 1);
    __syncthreads();
    const int item = s_item;
    if (item >= n_items) {
      if (!may_steal) break;
      if (others < 0) {
        // one parallel look at the other seven counters (they only grow, so
        // a queue seen exhausted stays exhausted)
        if (tid == 0) s_others = 0;
        __syncthreads();
        if (tid < 7) {
          const int x = (xcd + 1 + tid) & 7;
          const int c = __hip_atomic_load(g.counters + 8 * blockIdx.z + x, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
          if (c < queue_items(x)) atomicOr(&s_others, 1 << tid);
        }
        __syncthreads();
        others = s_others;
      }
      if (others == 0) break;
      const int i = __ffs(others) - 1;
      others &= others - 1;
      qx = (xcd + 1 + i) & 7;
      n_items = queue_items(qx);
      ctr = g.counters + 8 * blockIdx.z + qx;
      continue;
    }
    PairDesc P;
    int tile, chunk_id;
    bool shared = false;   // a shared tile of a batch (else a tile of one pair)
    if (!BATCH || g.pairs == nullptr) {
      P = g.one;
      const int m = item / P.n_tiles;
      tile = item - m * P.n_tiles;
      chunk_id = qx + 8 * m;
    } else {
      // the record holding this item, then the pair within its DM group
      const SuperChunk* rec = g.recs + g.rec_off[qx];
      int lo = 0, hi = g.rec_cnt[qx] - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rec[mid].item0 <= item) lo = mid; else hi = mid - 1;
      }
      const SuperChunk r = rec[lo];
      int local = item - r.item0;
      const int2 grp = g.groups[r.dm];
      if (g.jslots != nullptr) {
        // the DM-level fields (IF stack, actuators) are the group's first pair's
        shared = true;
        P = g.pairs[grp.x];
        tile = g.jgroups[r.dm].x + local;
      } else {
        int pi = grp.x;
        while (pi < grp.x + grp.y - 1 && local >= g.pairs[pi].n_tiles) {
          local -= g.pairs[pi].n_tiles;
          ++pi;
        }
        P = g.pairs[pi];
        tile = local;
      }
      chunk_id = r.chunk;
    }
    const int plane_bytes = P.H_in * P.W_in * 4;
    const size_t plane_in = (size_t)P.H_in * P.W_in;
    const int4 ti = shared ? g.jinfo[tile] : P.tile_info[tile];
    if (ti.y == 0) continue;   // empty tile
    // ti.w > 0: rows staged at that pitch from the tile's leftmost staged
    // column ti.z (IF pixel (y, x) at (y - y0) * pitch + x - ti.z), row table
    // (first, end) of each row's staged columns relative to ti.z;
    // else packed, ti.z floats, row table (first column, packed offset)
    const int y0 = ti.x, pitch = ti.w;
    const int nfl = pitch > 0 ? ti.y * pitch : ti.z;
    const int X0 = ti.z;
    // the tile's row table goes to LDS (one coalesced load), where the row
    // lookups below run without a memory round trip each
    {
      const int bhm = shared ? g.jBHmax : P.BHmax;
      const int2* rows_g = (shared ? g.jrows : P.rows) + (size_t)tile * bhm;
      for (int r = tid; r < bhm; r += BLOCK) s_rows[r] = rows_g[r];
    }
    // this lane's subaperture, and the pair it belongs to
    int kk;
    const int2* origin_l = P.origin;
    const int2* hrows_l = P.hrows;
    const float* weights_l = P.weights;
    float* out_l = P.out;
    int nv_l = P.nv;
    if (shared) {
      const int e = slot < g.jNS ? g.jslots[(size_t)tile * g.jNS + slot] : -1;
      kk = e < 0 ? -1 : (e & 0xFFFFF);
      if (e >= 0) {
        const PairDesc* L = g.pairs + (e >> 20);
        origin_l = L->origin;
        hrows_l = L->hrows;
        weights_l = L->weights;
        out_l = L->out;
        nv_l = L->nv;
      }
    } else {
      kk = slot < P.ns ? P.slot_kk[(size_t)tile * P.ns + slot] : -1;
    }
    const int2* rows = s_rows;

    int2 o = make_int2(0, 0), hr = make_int2(0, 0);
    if (kk >= 0) {
      o = origin_l[kk];
      hr = hrows_l[kk];
    }
    __syncthreads();   // the row table is in LDS
    int base[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      // patch rows outside [hr.x, hr.y) hold zero weights and need not be
      // staged: such a row reads the nearest one that is (finite values, and
      // the address of another lane of the subaperture, which the LDS
      // broadcasts instead of serialising a bank conflict)
      const int pr = min(max(q + LPS * i, hr.x), hr.y - 1);
      base[i] = 0;
      if (kk >= 0 && hr.x < hr.y) {
        const int r = o.y + pr - y0;
        base[i] = pitch > 0 ? r * pitch + (o.x - X0) : rows[r].y + (o.x - rows[r].x);
      }
    }

    // A stage holds KP consecutive actuators' packed tile rows (as many as
    // fit, up to KPMAX): small tiles then still fill the stage, which keeps
    // more useful bytes in flight per CU.  The actuators of a chunk are
    // taken in groups of KP; group gi is actuators a0 + gi*KP .. (< a1).
    const int cap_f = NJ * BLOCK * VW;
    const int KP = KPMAX == 1 || nfl == 0
                       ? 1
                       : max(1, min(min(KPMAX, cap_f / nfl), INT_MAX / plane_bytes));
    // byte offsets (within a group's KP consecutive actuator planes) of this
    // lane's DMA vectors; out-of-range offsets make the buffer unit return
    // zeros: vectors past the packed rows, outside the IF grid, or (via the
    // record count) of actuators past the end of the chunk
    unsigned voff[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int fo = (BLOCK * j + tid) * VW;   // float offset of the vector in the stage
      unsigned v = 0x80000000u;
      const int kp = KPMAX == 1 ? (fo < nfl ? 0 : 1) : (nfl > 0 ? fo / nfl : KP);
      if (kp < KP) {
        const int fr = fo - kp * nfl;          // offset within that actuator's rows
        int lo, gx;
        bool in_row = true;
        if (pitch > 0) {
          // rows at one pitch: vectors outside a row's staged columns are
          // not fetched
          lo = fr / pitch;
          const int c = fr - lo * pitch;
          in_row = lo < ti.y && c >= rows[lo].x && c < rows[lo].y;
          gx = X0 + c;
        } else {
          lo = 0;                              // last row whose offset is <= fr
          int hi = ti.y - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rows[mid].y <= fr) lo = mid; else hi = mid - 1;
          }
          gx = rows[lo].x + fr - rows[lo].y;
        }
        if (in_row) {
          const int gy = y0 + lo;
          if (gx >= 0 && gx + VW <= P.W_in && gy >= 0 && gy < P.H_in)
            v = (unsigned)kp * (unsigned)plane_bytes + (unsigned)(gy * P.W_in + gx) * 4u;
        }
      }
      voff[j] = v;
    }
    float wx[RPL][PW], wy[RPL][PW];
    if (kk >= 0) {
      const float* W = weights_l + ((size_t)plane * nv_l + kk) * 2 * E;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
#pragma unroll
        for (int c = 0; c < PW; ++c) {
          wx[i][c] = W[(q + LPS * i) * PW + c];
          wy[i][c] = W[E + (q + LPS * i) * PW + c];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int c = 0; c < PW; ++c) wx[i][c] = wy[i][c] = 0.f;
    }
    // chunk = P.chunk actuators, or (P.chunk == 0) an even split of the
    // actuators over P.n_chunks chunks
    const int a0 = P.chunk > 0 ? chunk_id * P.chunk
                               : (int)((long long)chunk_id * P.n_act / P.n_chunks);
    const int a1 = P.chunk > 0 ? min(P.n_act, a0 + P.chunk)
                               : (int)((long long)(chunk_id + 1) * P.n_act / P.n_chunks);
    const int n_grp = a1 > a0 ? (a1 - a0 + KP - 1) / KP : 0;
    // XCD sync (single pair only; E >= NST - 1 groups is guaranteed by the host)
    const bool sync_on = (!BATCH || g.pairs == nullptr) && g.sync_every > 0;
    const int sync_e = sync_on ? g.sync_every : 1;
    int* sync_ctr = g.sync_ctr + (8 * blockIdx.z + xcd) * SYNC_STRIDE;
    bool sync_live = true;

    auto consume = [&](const float4* buf, int gi) {
      const float* fb = reinterpret_cast<const float*>(buf);
#pragma unroll
      for (int kp = 0; kp < KPMAX; ++kp) {
        if (kp >= KP) break;
        const int a = a0 + gi * KP + kp;
        const bool act = a < a1;
        const float* fk = fb + kp * nfl;
        float sx = 0.f, sy = 0.f;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          if constexpr (BATCH || PW >= 12) {
            // a row's values are all read before its products, so that its
            // LDS reads are in flight together (left alone, the scheduler
            // may issue each read just ahead of its two products and wait for
            // it there, one LDS latency per pair of values).  The batch, and
            // wide patches (rotated or magnified maps), are bound by this
            // contraction; the narrower single-pair patches hide it behind
            // the DMA and keep the compiler's order, which needs fewer
            // registers.
            float f[PW];
#pragma unroll
            for (int c = 0; c < PW; ++c) f[c] = fk[base[i] + c];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < PW; ++c) {
              sx = __fmaf_rn(wx[i][c], f[c], sx);
              sy = __fmaf_rn(wy[i][c], f[c], sy);
            }
          } else {
#pragma unroll
            for (int c = 0; c < PW; ++c) {
              const float f = fk[base[i] + c];
              sx = __fmaf_rn(wx[i][c], f, sx);
              sy = __fmaf_rn(wy[i][c], f, sy);
            }
          }
        }
        sx = dpp_sum(sx, LPS);
        sy = dpp_sum(sy, LPS);
        const size_t row = (size_t)(act ? a : a0) * 2 * nv_l;
        if (VJP) {
          if (act && kk >= 0 && q == 0)
            vacc += (double)g.grad[row + kk] * sx + (double)g.grad[row + nv_l + kk] * sy;
        } else {
          // exactly one store instruction per wave and actuator slot, whatever
          // the lanes hold (the pipeline's wait counts rely on this number).
          // Every lane of a subaperture holds both sums after the DPP
          // reduction: even lanes store s_x, odd lanes s_y, so the extra
          // lanes repeat a real store (same address, same value) and add no
          // memory traffic.  Only empty slots and the slots past the chunk's
          // end target a scratch slot.
          float* o = out_l + (size_t)(plane - g.out_plane0) * P.n_act * 2 * nv_l + row;
          const bool real = act && kk >= 0;
          const bool ycomp = (q & 1) != 0;
          float* dst = real ? (ycomp ? o + nv_l + kk : o + kk) : g.scratch + (tid & 63);
          const float val = ycomp ? sy : sx;
          // a global (not flat) store: flat operations may complete out of
          // order with the DMA, and the wait counts need them in order.  A
          // plain (write-back) store: the pieces that the tiles of one chunk
          // write into an IM row merge in the XCD's L2, and the scratch slot
          // stays there (streaming stores measured 4% slower on the ELT build)
          *(gfloat_t*)dst = val;
        }
      }
    };
    // Loads group gi into stage k.  With the XCD sync on, lane 0 first adds
    // the workgroup's entry when gi opens a block, then snapshots the counter
    // into s_snap[k]; both precede the stage's DMA.
    auto issue = [&](int k, float4* buf, int gi) {
      if (sync_on && tid == 0) {
        if (gi % sync_e == 0) atomicAdd(sync_ctr, 1);
        snapshot_issue(sync_ctr, s_snap + k);
      }
      const int a = a0 + gi * KP;
      const int cnt = min(KP, a1 - a);
      stage_issue<BLOCK, NJ, VW>(P.ifs + (size_t)a * plane_in, cnt * plane_bytes, voff, buf,
                                 wave);
    };
    // one pipeline step for group gi held in stage K: wait for it (the later
    // stages already issued may stay in flight), make it visible to every
    // wave, refill the stage freed by the previous step with group gi+NST-1,
    // then consume.  Vector-memory operations complete in issue order, so
    // "at most n in flight", n = the operations issued after this stage's
    // DMA, means this stage has landed.  The wait counts every
    // vector-memory operation issued after this stage's DMA: the later
    // stages' DMA (NJ each) and, in the IM kernel, the KP stores of each step
    // since then.
    //
    // With the XCD sync on, group j with j a multiple of E opens block j/E,
    // and a workgroup may open block b >= 1 only once every tile of its XCD
    // has opened block b - 1 (counter >= b * n_part).  Wave 0 checks the
    // snapshot that came with the stage just waited for; only if that is
    // short does it poll the counter itself (bounded: a workgroup that waits
    // too long stops waiting but keeps adding its entries, so the counts stay
    // exact).  Wave 0 also issues, per loaded group, the snapshot and
    // possibly an entry atomic; its wait counts them.
    auto step = [&](auto kc, int gi) {
      constexpr int K = decltype(kc)::value;
      const int later = min(NST - 2, n_grp - 1 - gi);
      const int stores = VJP ? 0 : KP * min(gi, NST - 1);
      const int x = gi + NST - 1;   // the group this step starts loading
      int extra = 0;
      if (sync_on && wave == 0) extra = later + (gi + later) / sync_e - gi / sync_e;
      wait_vm(later * NJ + stores + extra);
      if (sync_on && wave == 0 && sync_live && x < n_grp && x > 0 && x % sync_e == 0) {
        const int target = (x / sync_e) * n_part;
        if (s_snap[K] < target) {
          int it = 0;
          while (__hip_atomic_load(sync_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                 target) {
            if (++it >= SYNC_SPIN_MAX) {
              sync_live = false;
              break;
            }
            __builtin_amdgcn_s_sleep(4);
          }
        }
      }
      stage_barrier();
      if (x < n_grp) issue((K + NST - 1) % NST, stage_buf<(K + NST - 1) % NST, STAGE_F4>(), x);
      consume(stage_buf<K, STAGE_F4>(), gi);
    };
    // every compiler-tracked load of the item (weights, rows) has landed
    // before the first DMA; otherwise the compiler would wait for them at
    // their first use inside the pipeline, with vmcnt(0), draining the DMA
    // queue at every loop head.
    wait_vm(0);
    [&]<int... K>(std::integer_sequence<int, K...>) {
      ((K < n_grp && K < NST - 1 ? issue(K, stage_buf<K, STAGE_F4>(), K) : void()), ...);
    }(std::make_integer_sequence<int, NST>{});
    for (int gb = 0; gb < n_grp; gb += NST) {
      [&]<int... K>(std::integer_sequence<int, K...>) {
        ((gb + K < n_grp ? step(std::integral_constant<int, K>{}, gb + K) : void()), ...);
      }(std::make_integer_sequence<int, NST>{});
    }
  }
  wait_vm(0);   // no DMA or store of this workgroup outlives it
  if (VJP) {
    // fixed-order reduction: butterfly within each wave, then over the waves
    double v = vacc;
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) s_red[wave] = v;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < BLOCK / 64; ++w) s += s_red[w];
      g.partials[(size_t)(plane - 1) * gridDim.x + blockIdx.x] = s;
    }
  }
  if (g.finish != nullptr) {
    // Every workgroup has taken its last item before it counts itself
    // finished: its counter operations are device-scope atomics whose
    // results it waited for, so they are performed before its finish count.
    // The last one clears the counters with plain stores, which the end of
    // the kernel makes visible to the next launch.  (No fence: a device-scope
    // release here would write back the XCD's L2 at every workgroup's exit.)
    __shared__ int s_last;
    __syncthreads();
    if (tid == 0)
      s_last = atomicAdd(g.finish, 1) == (int)(gridDim.x * gridDim.y * gridDim.z) - 1;
    __syncthreads();
    if (s_last) {
      for (int i = tid; i < g.n_counters; i += BLOCK) g.counters[i] = 0;
      if (tid == 0) *g.finish = 0;
    }
  }
}


// ------------------------------------------------------------------- variants

using StreamFn = void (*)(StreamArgs);


struct Variant {
  int BLOCK, LPS, RPL, PW, NJ4, NST;   // NJ4: 16-byte DMA instructions per wave per stage
  int PACK;                            // most actuators one stage holds
  StreamFn im4, vjp4;                  // 16-byte DMA: rows a multiple of 4 floats, aligned stack
  StreamFn im1, vjp1;                  // 4-byte DMA: any row length / alignment
  StreamFn bim4, bim1;                 // batched launches (IM only)
  int PH() const { return LPS * RPL; }
  int cap_floats() const { return NJ4 * BLOCK * 4; }
};

// 4-byte DMA issues 4x the instructions per stage: cap its depth to what the
// vmcnt counter can express
constexpr int nst_vw1(int n, int s) { return s < 2 + 63 / (4 * n) ? s : 2 + 63 / (4 * n); }

#define SYNIM_VARIANT_K(B, L, R, W, N, S, K)                                           \
  {B, L, R, W, N, S, stage_pack(N, S, K),                                              \
   im_stream_kernel<B, L, R, W, N, 4, S, K, false, false>,                             \
   im_stream_kernel<B, L, R, W, N, 4, S, K, true, false>,                              \
   im_stream_kernel<B, L, R, W, 4 * N, 1, nst_vw1(N, S), K, false, false>,             \
   im_stream_kernel<B, L, R, W, 4 * N, 1, nst_vw1(N, S), K, true, false>,              \
   im_stream_kernel<B, L, R, W, N, 4, S, K, false, true>,                              \
   im_stream_kernel<B, L, R, W, 4 * N, 1, nst_vw1(N, S), K, false, true>}
#define SYNIM_VARIANT(B, L, R, W, N, S) SYNIM_VARIANT_K(B, L, R, W, N, S, 1)
#define SYNIM_VARIANT_PACK(B, L, R, W, N, S) SYNIM_VARIANT_K(B, L, R, W, N, S, 4)

// Parts of the variant table (one per translation unit, in table order).
constexpr int kVariantParts = 8;
const Variant* stream_variants_0(int* n);
const Variant* stream_variants_1(int* n);
const Variant* stream_variants_2(int* n);
const Variant* stream_variants_3(int* n);
const Variant* stream_variants_4(int* n);
const Variant* stream_variants_5(int* n);
const Variant* stream_variants_6(int* n);
const Variant* stream_variants_7(int* n);

}  // namespace synim
