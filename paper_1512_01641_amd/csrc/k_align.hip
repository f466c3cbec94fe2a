// Needleman-Wunsch global alignment of the sentence sequences of every
// document pair (Sec. 5.1, Figs. 1-2, eq. (1)) and the threshold filter
// (Sec. 4).
//
// k_nw_fill   persistent work-queue kernel, four waves per workgroup.  A
//             strip is 64 rows of one pair's DP lattice; a task is four
//             strips, one per wave: four consecutive strips of one pair (fewer
//             at its end) or strips of one-strip pairs, in queue order
//             (longest chains first).  Lane r owns row r of the strip and at
//             step t computes column j = t - r + 1, so each step is one
//             anti-diagonal of the strip, computed by all lanes at once
//             (Sec. 5.1, Fig. 2).  Per cell, in FP32 without contraction:
//                up = H[i-1][j] + g, left = H[i][j-1] + g, diag = H[i-1][j-1] + S
//                first maximum of (up, left, diag) with '>' (UP > LEFT > DIAG)
//             The value from the row above moves one lane per step by a DPP
//             wave shift.  The strip's top boundary (the previous strip's last
//             row) enters lane 0 through a 64-lane register window shifted one
//             lane per step; the strip's own last row leaves through a second
//             shifted window every 16 steps.  Between the strips of one task
//             the row passes through an LDS ring with a count of columns put
//             and taken (about 80 steps behind); the last strip of a task
//             publishes it as tagged 64-bit agent-coherent stores (no
//             counters, no cache flushes) for the first strip of the next
//             task, which runs on another workgroup about 150 steps behind
//             (bounded re-read).  A wave that gives up waiting (its poll
//             limit) sets the error flag, marks its own last row failed (tag
//             TAG_FAIL in memory, count -1 in LDS, so the strips below give up
//             at once instead of waiting out their own limits) and, in a
//             pair's last strip, writes NaN as the score; the walk then leaves
//             the pair empty.  S is staged through an LDS ring of two 64-step
//             groups per wave (16 KiB each: 64 rows x 256 bytes), filled a
//             group ahead by 16-byte LDS-direct buffer loads (no register
//             holds S); each lane reads the four steps of one 16-byte chunk
//             of its own row with one ds_read_b128, placed so that the lanes
//             of a quarter-wave hit different banks.  Each lane packs its
//             2-bit directions, 16 steps per word, and every 64 steps the
//             wave writes one coalesced 1 KiB block.  H never reaches HBM.
// k_nw_reset  clears the published-row region and the queue; scores of
//             empty pairs.
// k_nw_walk   traceback from (n, m): one wave per pair holds one 64-step
//             block of its strip (one 16-byte word per lane) and reads it with
//             uniform-index readlane, with the previous block prefetched.
//             Aligned pairs are written right-aligned (ascending) into the
//             path area.
// k_keep      keeps the aligned pairs with S >= threshold, ascending.
#include "nwm_internal.h"

#include <algorithm>
#include <cmath>

namespace nwm {

constexpr int GROUP = 64;             // steps per S staging group (four chunks of 16)
constexpr int GROUP_FLOATS = 64 * GROUP;   // ring floats per group (64 rows x 256 bytes)
constexpr int RING_GROUPS = 2;        // groups in the S ring: one in flight while one is read
constexpr int SPIN_LIMIT = 1 << 22;   // default polls before a wave gives up (error flag)
constexpr uint32_t TAG_FAIL = 2u;     // tag of a boundary value whose producer gave up

static __device__ __forceinline__ float dpp_shr1(float old, float src) {
  // lane l <- src of lane l-1; lane 0 keeps `old`
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), 0x138, 0xF, 0xF, false));
}
static __device__ __forceinline__ float dpp_shl1(float old, float src) {
  // lane l <- src of lane l+1; lane 63 keeps `old`
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), 0x130, 0xF, 0xF, false));
}

static __device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// A 64-bit value every lane holds the same value of, moved to scalar registers.
static __device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A pointer every lane holds the same value of, moved to scalar registers.
template <typename T>
static __device__ __forceinline__ T *uniform_ptr(T *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

// The parallelogram of S used by steps [GROUP*q, GROUP*q + GROUP): row r,
// columns GROUP*q - r + [0, GROUP), 256 bytes per row.  It goes straight
// from memory into one ring slot of 16 KiB by 16 LDS-direct 16-byte buffer
// loads; load k brings rows 4k .. 4k + 3 into the slot's k-th KiB.  Within
// that KiB, lane l of the load writes bytes 16 l .. 16 l + 15, so the lane
// that loads 16-byte chunk c (steps 4c .. 4c + 3) of row 4k + rho is the
// one that puts it where the reader wants it:
//    lane = 16 rho + ((c + 4 (k & 3) + rho) & 15).
// Every lane of the reader (lane = row) then reads chunk c of its own row
// with one ds_read_b128, and the 16 lanes of each quarter-wave (rows
// 16p + j) fall on 16 different 16-byte bank groups ((c + j) & 15).  The 16
// lanes of a load that share rho read one row's 256 contiguous bytes.  No
// register holds S.
//
// Lane l of load k reads strip bytes 4 (r (m - 1) + GROUP q) + 16 c for its
// row r = 4k + rho and chunk c: base_{k & 3} + (k >> 2) 64 (m - 1) + 256 q,
// with the group offset in the VGPR offset so that the range check covers it.
// A cell outside the strip's m columns (the first steps of a row, the steps
// after its last column) reads another cell of the strip, or 0 past the
// strip's end through the buffer range check: a value that only the masked
// steps see, and those leave H unchanged there.  Rows at or beyond `rows`
// (the last strip of a pair) lie past the end.  Groups past the strip's
// last step are loaded from an offset past the range (no memory access), so
// every group issues the same 16 loads.
struct StripSrc {
  __amdgpu_buffer_rsrc_t rs;
  uint32_t base[4];        // bytes, this lane's (row, chunk) in loads 0..3
  uint32_t step;           // bytes from load k to load k + 4: 64 (m - 1)
  int n_groups;            // groups holding steps of the strip
};

typedef __attribute__((address_space(3))) void lds_void;

typedef unsigned int u32x2v __attribute__((ext_vector_type(2)));
constexpr int CPOL_SC1 = 16;          // cache-policy bit of an agent-coherent access
constexpr int PUB_NONE = 0x40000000;  // buffer offset past any boundary row: the store is dropped

// The strip's last row: one tagged 64-bit agent-coherent store per lane into
// the boundary row `rs` (slot j at byte 8 j).  Every lane issues the store, so
// each chunk issues the same memory operations; a lane with nothing to
// publish stores at PUB_NONE, past the buffer's range, and the range check
// drops it without a memory access.
static __device__ __forceinline__ void publish(__amdgpu_buffer_rsrc_t rs, bool pub, int j, uint64_t v) {
  const u32x2v d = {(uint32_t)v, (uint32_t)(v >> 32)};
  __builtin_amdgcn_raw_buffer_store_b64(d, rs, pub ? 8 * j : PUB_NONE, 0, CPOL_SC1);
}

constexpr uint32_t S_NONE = 0x40000000u;   // buffer offset past any strip (S stays below 1 GiB per strip)

// The lane's byte base for load j < 4 (see StripSrc): row rho of the load
// and chunk c, inverting lane = 16 rho + ((c + 4 j + rho) & 15).
static __device__ __forceinline__ uint32_t s_lane_base(int lane, int j, int m) {
  const int rho = lane >> 4;
  const int c = ((lane & 15) - 4 * j - rho) & 15;
  return (uint32_t)(4 * j + rho) * (uint32_t)(m - 1) * 4u + 16u * (uint32_t)c;
}

#define NWM_S_LOAD(A)                               \
  "buffer_load_dwordx4 " A ", %9, 0 offen lds\n\t"  \
  "s_add_u32 m0, m0, 1024\n\t"                      \
  "v_add_u32 " A ", %10, " A "\n\t"
#define NWM_S_LOAD4 NWM_S_LOAD("%1") NWM_S_LOAD("%2") NWM_S_LOAD("%3") NWM_S_LOAD("%4")

// The 16 loads of group q into ring slot `slot`, in one asm statement so that
// the compiler neither reorders them with other memory accesses nor adds
// waits for them: every read of the ring waits for them with an explicit
// vmcnt (below).  M0 (the LDS address of a load) is saved, stepped by 1 KiB
// per load and restored; a VALU instruction separates each M0 write from the
// load that uses it.
static __device__ __forceinline__ void load_group(float *ring, const StripSrc &src, int q, int slot) {
  const uint32_t la = (uint32_t)uniform((int)(uint32_t)(uintptr_t)(lds_void *)(ring + slot * GROUP_FLOATS));
  const uint32_t goff = (uint32_t)uniform(q < src.n_groups ? (int)(GROUP * 4 * q) : (int)S_NONE);
  uint32_t save, a0, a1, a2, a3;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %5\n\t"
      "v_add_u32 %1, %8, %6\n\t"
      "v_add_u32 %2, %8, %7\n\t"
      "v_add_u32 %3, %8, %11\n\t"
      "v_add_u32 %4, %8, %12\n\t"
      NWM_S_LOAD4 NWM_S_LOAD4 NWM_S_LOAD4 NWM_S_LOAD4
      "s_mov_b32 m0, %0"
      : "=&s"(save), "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3)
      : "s"(la), "v"(src.base[0]), "v"(src.base[1]), "s"(goff), "s"(src.rs), "s"(src.step), "v"(src.base[2]),
        "v"(src.base[3])
      : "memory", "scc");
}
#undef NWM_S_LOAD4
#undef NWM_S_LOAD

// One 16-byte agent-coherent (sc1) LDS-direct load per active lane: lane l
// writes bytes 16 l .. 16 l + 15 of buf.  Written as asm for the same reason
// as the S loads: the compiler's own tracking of an LDS-direct load makes
// every later LDS read (the ring included) wait for all loads in flight,
// which would cancel the two-group prefetch.  Its readers wait with an
// explicit vmcnt.  One wait state separates the M0 write from the load.
static __device__ __forceinline__ void load_window_lds(uint64_t *buf, const uint64_t *src) {
  const uint32_t la = (uint32_t)uniform((int)(uint32_t)(uintptr_t)(lds_void *)buf);
  uint32_t save;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %2, off sc1\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(save)
      : "s"(la), "v"(src)
      : "memory");
}

struct StripState {
  float H, diag, pw, col;
  uint32_t bits;
};

// 16 steps starting at t0 (a multiple of 16).  MASKED chunks (the first 64
// steps and the steps past column m) update H only where 1 <= j <= m, so a
// lane keeps H[i][0] until its column starts and keeps H[i][m] after it ends;
// in between every lane is active.  Every step also shifts the last-row
// collector (lane 63 enters), used by strips that have a successor.
//
// MAX3: the new H is max(up, left, diag) in one instruction, and the
// direction (the first of up, left, diag equal to it) is found off the
// dependency chain from one step to the next.  This is the first maximum
// with '>' bit for bit whenever no operand is NaN or -0: a finite S and a gap
// that is not -0 never produce either (H starts at +0 or i*gap != 0, and a
// sum is -0 only when both terms are).  A gap of -0 takes the compare chain.
template <bool MASKED, bool MAX3>
static __device__ __forceinline__ void run16v(StripState &st, const float4 (&sv)[4], int t0, int m, float g,
                                              int lane) {
  float H = st.H, diag = st.diag, pw = st.pw, col = st.col;
  uint32_t bits = 0;
  int d = t0 - lane;   // column - 1 of this lane at the current step
  // MAX3: the direction of a step is packed during the next one
  float up_p = 0.0f, left_p = 0.0f, best_p = 0.0f;
  auto code3 = [](float up, float left, float best) -> uint32_t {
    return up == best ? (uint32_t)DIR_UP : (left == best ? (uint32_t)DIR_LEFT : (uint32_t)DIR_DIAG);
  };
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const float4 v4 = sv[u >> 2];
    const float s = (u & 3) == 0 ? v4.x : (u & 3) == 1 ? v4.y : (u & 3) == 2 ? v4.z : v4.w;
    const float x = dpp_shr1(pw, H);   // H[i-1][j]: lane r-1, or the boundary row for lane 0
    const float up = x + g;
    const float left = H + g;
    const float dg = diag + s;
    float best;
    if (MAX3) {
      best = __builtin_fmaxf(__builtin_fmaxf(up, left), dg);
      if (u > 0) {
        bits = (bits << 2) | code3(up_p, left_p, best_p);
        asm volatile("" : "+v"(bits));
      }
      up_p = up;
      left_p = left;
      best_p = best;
    } else {
      const bool c1 = left > up;
      const float b1 = c1 ? left : up;
      const bool c2 = dg > b1;
      best = c2 ? dg : b1;
      bits = (bits << 2) | (c2 ? (uint32_t)DIR_DIAG : (c1 ? (uint32_t)DIR_LEFT : (uint32_t)DIR_UP));
      asm volatile("" : "+v"(bits));   // pack now: do not keep 16 steps of compare masks alive
    }
    if (MASKED) {
      H = ((unsigned)d < (unsigned)m) ? best : H;
      ++d;
    } else {
      H = best;
    }
    diag = x;
    pw = dpp_shl1(pw, pw);
    col = dpp_shl1(H, col);
    if (!MAX3) __builtin_amdgcn_sched_barrier(0);   // one step at a time
  }
  if (MAX3) bits = (bits << 2) | code3(up_p, left_p, best_p);
  st.H = H;
  st.diag = diag;
  st.pw = pw;
  st.col = col;
  st.bits = bits;
}

// The float offset, within a ring slot, of chunk c (steps 4c .. 4c + 3) of
// row `lane` (see StripSrc).
static __device__ __forceinline__ uint32_t chunk_off(int lane, int c) {
  return (uint32_t)(256 * (lane >> 2) + 4 * (16 * (lane & 3) + ((c + 4 * ((lane >> 2) & 3) + (lane & 3)) & 15)));
}

// The 16 S values of lane `lane` for the steps [t0, t0 + 16) from the ring
// slot `grp`; `off` holds the lane's offsets of the four chunks.
template <bool MASKED, bool MAX3>
static __device__ __forceinline__ void run16(StripState &st, const float *grp, const uint32_t (&off)[4], int t0,
                                             int m, float g, int lane) {
  float4 sv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) sv[q] = *reinterpret_cast<const float4 *>(grp + off[q]);
  run16v<MASKED, MAX3>(st, sv, t0, m, g, lane);
}

struct FillArgs {
  int n_items, B;
  int item0;        // first work item of this launch (its queue counts from 0)
  int n_tasks;      // tasks of this launch (the LDS-ring fill)
  int task0;        // its first task
  int spin_limit;   // polls of a boundary window before the wave gives up
  int hold;         // testing: the first strip of a pair publishes nothing
  const int32_t *it_pair, *it_strip, *n, *m;
  const int32_t *tk_pair, *tk_slot;
  const int64_t *s_off, *tb_off, *bnd_off;
};

// LDS of the LDS-ring fill, per workgroup of SLOTS waves: each wave's S
// ring and window buffers, then a link ring per pair of neighbouring waves
// (the upper strip's last row, LINK_COLS columns, column j in slot
// j % LINK_COLS), then the counters: [k] columns wave k has put into link k
// (-1: it gave up), [SLOTS + k] columns wave k + 1 has taken from it,
// [2 SLOTS] the task.  SLOTS = 1: one strip per workgroup, no links.
constexpr int FILL_WAVE_LDS = RING_GROUPS * GROUP_FLOATS * 4 + 2 * 32 * 8;
constexpr int LINK_COLS = 512;
constexpr int fill_lds_bytes(int slots) {
  return slots * FILL_WAVE_LDS + (slots - 1) * LINK_COLS * 4 + 4 * (2 * slots + 1);
}
static_assert((LINK_COLS & (LINK_COLS - 1)) == 0 && LINK_COLS >= 256, "link ring");

__global__ __launch_bounds__(256) void k_nw_reset(FillArgs A, uint4 *__restrict__ bnd16, int64_t n_bnd16,
                                                  int32_t *__restrict__ ctl, float g, float *__restrict__ score) {
  const int64_t tid = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * 256;
  // published boundary values carry tag 1; clearing them every launch means a
  // value left by an earlier launch is never taken as ready
  for (int64_t k = tid; k < n_bnd16; k += nthr) bnd16[k] = make_uint4(0u, 0u, 0u, 0u);
  if (tid < 4) ctl[tid] = 0;   // [0] queue head, [1] error flag, [2] queue head of a second launch
  for (int64_t b = tid; b < A.B; b += nthr) {
    const int n = A.n[b], m = A.m[b];
    // H[n][0] = fl32(n*g), H[0][m] = fl32(m*g), H[0][0] = +0
    if (n == 0 || m == 0) score[b] = (n + m == 0) ? 0.0f : (float)(n + m) * g;
  }
}

template <bool MAX3, int SLOTS>
__global__ __launch_bounds__(64 * SLOTS) void k_nw_fill(FillArgs A, const float *__restrict__ S, float g,
                                                        float *__restrict__ score, char *__restrict__ tb,
                                                        uint64_t *__restrict__ bnd, int32_t *__restrict__ head,
                                                        int32_t *__restrict__ err) {
  constexpr uint32_t epoch = 1u;   // tag of a published value (the reset clears to 0)
  extern __shared__ __align__(16) char fill_lds[];   // fill_lds_bytes(SLOTS) bytes
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float *ring = reinterpret_cast<float *>(fill_lds + wave * FILL_WAVE_LDS);
  uint64_t *winbufA = reinterpret_cast<uint64_t *>(fill_lds + wave * FILL_WAVE_LDS + RING_GROUPS * GROUP_FLOATS * 4);
  uint64_t *winbufB = winbufA + 32;   // boundary windows (LDS-direct loads)
  float *links = reinterpret_cast<float *>(fill_lds + SLOTS * FILL_WAVE_LDS);
  int *ctr = reinterpret_cast<int *>(fill_lds + SLOTS * FILL_WAVE_LDS + (SLOTS - 1) * LINK_COLS * 4);
  float *link_in = links + (wave - 1) * LINK_COLS;   // from the wave above (wave > 0)
  float *link_out = links + wave * LINK_COLS;        // to the wave below (wave < SLOTS - 1)
  // this lane's ring offsets of the four 16-byte chunks of each 16 steps of
  // a group
  uint32_t off[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) off[i][c] = chunk_off(lane, 4 * i + c);
  // One task (SLOTS strips, one per wave) at a time: the whole
  // workgroup takes the next task once every wave is done with the last one,
  // so the link rings and counters start clear.  Every wave passes both
  // barriers of every task and leaves the loop at the same task.
  for (;;) {
    __syncthreads();
    if (threadIdx.x < 2 * SLOTS) ctr[threadIdx.x] = 0;
    if (threadIdx.x == 0) ctr[2 * SLOTS] = atomicAdd(head, 1);
    __syncthreads();
    const int task = uniform(ctr[2 * SLOTS]);
    if (task >= A.n_tasks) break;
    const int ts = (A.task0 + task) * SLOTS + wave;   // this wave's task slot
    const int b = uniform(A.tk_pair[ts]);
    if (b < 0) continue;   // an empty slot
    const int s_tag = uniform(A.tk_slot[ts]);
    const int s = s_tag & ITEM_STRIP;
    const bool hot = (s_tag & ITEM_HOT) != 0;
    const bool link_up = (s_tag & ITEM_LINK_IN) != 0;     // the boundary comes from the wave above, in LDS
    const bool link_down = (s_tag & ITEM_LINK_OUT) != 0;  // the last row goes to the wave below, in LDS
    const bool in_global = s > 0 && !link_up;             // the boundary comes from memory
    if (hot) __builtin_amdgcn_s_setprio(2);
    const int n = uniform(A.n[b]), m = uniform(A.m[b]);
    const int nstrips = (n + 63) >> 6;
    const bool last = s == nstrips - 1;
    const int i0 = 64 * s;
    const int rows = min(64, n - i0);
    const float *Sb = S + A.s_off[b];
    const int64_t mstride = bnd_stride(m);
    const int64_t bnd_off = uniform64(A.bnd_off[b]), tb_off = uniform64(A.tb_off[b]);
    const uint64_t *in_row = bnd + bnd_off + (int64_t)(s - 1) * mstride;   // used when s > 0
    uint64_t *out_row = bnd + bnd_off + (int64_t)s * mstride;               // used when !last
    const int nG = (m + 63 + 63) >> 6;
    uint4 *tbs = reinterpret_cast<uint4 *>(tb + tb_off) + (int64_t)s * nG * 64;
    const int T_end = m + rows - 1;
    const int T_pad = (T_end + 15) & ~15;
    const int r_last = n - 1 - i0;   // lane of row n in the last strip
    bool failed = false;

    // slots 1..m of this strip's published row (nothing when it is the last
    // or hands its row on through LDS: the store instruction still issues)
    const __amdgpu_buffer_rsrc_t pub_rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)uniform_ptr(out_row), (short)0, (last || link_down) ? 0 : uniform((m + 1) * 8), 0x00020000);

    StripSrc src;
    src.rs = __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(Sb + (int64_t)i0 * m), (short)0,
                                               uniform(rows * m * 4), 0x00020000);
#pragma unroll
    for (int j = 0; j < 4; ++j) src.base[j] = s_lane_base(lane, j, m);
    src.step = (uint32_t)uniform(64 * (m - 1));
    src.n_groups = (T_pad + GROUP - 1) / GROUP;

    StripState st;
    const int i = i0 + 1 + lane;
    st.H = (float)i * g;                                    // H[i][0]
    st.diag = (i0 == 0) ? 0.0f : (float)i0 * g;             // lane 0: H[i0][0]
    st.col = 0.0f;
    st.bits = 0u;
    st.pw = 0.0f;

    // The pair's offsets are pinned in scalar registers before the S
    // prologue: a wait for them placed after it would also wait for its loads.
    asm volatile("" ::"s"(bnd_off), "s"(tb_off));

    // Boundary window prev[tw + 1 + lane]: the first row, or the previous
    // strip's last row published by another wave.  Every published value is
    // one 64-bit agent-coherent (sc1) store of (value, tag 1) into memory the
    // reset kernel cleared, so a consumer knows a value is there when its tag
    // is set: no counters, no store drains and no cache flushes.  Windows
    // are prefetched two chunks ahead straight into LDS (16-byte agent-coherent
    // LDS-direct loads, slots tw .. tw + 63), so no register holds a load in
    // flight; the wait for one is an explicit vmcnt over the fixed sequence of
    // memory operations of a group (below).
    // A reload waits for its value inside the same asm statement: a load the
    // compiler tracked could still be in flight where the spin loop rejoins
    // the sweep, and the compiler would then drain every load in flight (the
    // S prefetch included) before each later chunk.  The reload drains the
    // counter too, but only on this slow path.
    auto load_window = [&](int tw) -> uint64_t {
      uint64_t v;
      asm volatile(
          "global_load_dwordx2 %0, %1, off sc1\n\t"
          "s_waitcnt vmcnt(0)"
          : "=&v"(v)
          : "v"(in_row + tw + 1 + lane)
          : "memory");
      return v;
    };
    // lanes 0..8 bring slots tw .. tw + 17 (16 bytes each), which hold the
    // 16 values a chunk uses
    auto prefetch_window = [&](int tw, uint64_t *buf) {
      if (lane < 9) load_window_lds(buf, in_row + tw + 2 * lane);
    };
    // slot tw + 1 + lane of a window buffer (lanes 0..15 matter)
    const int wslot = 1 + (lane & 15);
    // lanes 0..15 feed the next 16 steps; columns beyond m are never used
    auto window_need = [&](int tw) -> bool { return lane < 16 && tw + 1 + lane <= m; };
    auto window_ready = [&](uint64_t v, int tw) -> bool {
      return __ballot(window_need(tw) && (uint32_t)(v >> 32) != epoch) == 0;
    };
    // the producer has not got this far yet: reload (bounded) until it has;
    // a value tagged TAG_FAIL means the producer gave up
    auto wait_window = [&](int tw, uint64_t v) -> uint64_t {
      int spins = 0;
      for (;;) {
        const uint32_t tag = (uint32_t)(v >> 32);
        if (__ballot(window_need(tw) && tag == TAG_FAIL) != 0) {
          failed = true;
          break;
        }
        if (__ballot(window_need(tw) && tag != epoch) == 0) break;
        if (++spins > A.spin_limit) {
          failed = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = load_window(tw);
      }
      return v;
    };
    // A bounded wait on a link counter (LDS, written by another wave of the
    // workgroup) until it reaches `need`; `seen` keeps the last value read,
    // so most chunks need no read at all.  False if the writer gave up (-1)
    // or the poll limit passed.  LDS accesses only: no vector memory counts.
    // A wave's LDS operations are performed in order, so a count written
    // after its values (or after the reads of the slots it frees) is never
    // seen before them; only the compiler is kept from reordering.
    auto link_wait = [&](const int *c, int need, int &seen) -> bool {
      for (int spins = 0; seen < need; ++spins) {
        if (spins > A.spin_limit) return false;
        if (spins > 0) __builtin_amdgcn_s_sleep(1);
        seen = uniform(__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (seen < 0) return false;
      }
      return true;
    };
    int up_put = 0;      // columns the wave above had put, as last read
    int down_taken = 0;  // columns the wave below had taken, as last read
    // the boundary of the 16 steps from tw, columns tw + 1 .. tw + 16, from
    // the wave above; then the columns taken are counted
    auto link_take = [&](int tw) -> uint64_t {
      if (!link_wait(&ctr[wave - 1], min(tw + 16, m), up_put)) {
        failed = true;
        return 0ull;
      }
      asm volatile("" ::: "memory");
      const float v = link_in[(tw + 1 + (lane & 15)) & (LINK_COLS - 1)];
      asm volatile("" ::: "memory");
      if (lane == 0)
        __hip_atomic_store(&ctr[SLOTS + wave - 1], tw + 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return ((uint64_t)epoch << 32) | __float_as_uint(v);
    };
    // the columns of the strip's last row finished in the chunk at t0 (lanes
    // 48.. of the collector) to the wave below, once it has taken what they
    // overwrite; then the count of columns put
    auto link_put = [&](int t0) {
      const int jhi = min(t0 - 47, m);
      if (jhi < 1 || (A.hold && s == 0)) return;
      if (!link_wait(&ctr[SLOTS + wave], jhi - LINK_COLS, down_taken)) {
        failed = true;
        return;
      }
      const int j = t0 - 110 + lane;
      if (lane >= 48 && j >= 1 && j <= m) link_out[j & (LINK_COLS - 1)] = st.col;
      asm volatile("" ::: "memory");
      if (lane == 0) __hip_atomic_store(&ctr[wave], jhi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // One chunk of 16 steps from its boundary window.  The publish of the
    // strip's last row is one store instruction in every chunk (see
    // publish), so the explicit wait counts stay exact.
    auto chunk = [&](int t0, uint64_t win, const float *grp, const uint32_t(&off)[4]) {
      st.pw = s > 0 ? __uint_as_float((uint32_t)win) : (float)(t0 + 1 + lane) * g;
      if (t0 < 64 || t0 + 16 > m) run16<true, MAX3>(st, grp, off, t0, m, g, lane);
      else run16<false, MAX3>(st, grp, off, t0, m, g, lane);
      // lane l of the collector holds H of row 64 at step t0 + 15 - 63 + l,
      // i.e. column t0 - 110 + l; lanes 48.. publish
      const int j = t0 - 110 + lane;
      const bool pub = !last && !link_down && lane >= 48 && j >= 1 && j <= m && !(A.hold && s == 0);
      publish(pub_rs, pub, j, ((uint64_t)epoch << 32) | __float_as_uint(st.col));
      if (link_down) link_put(t0);
      return st.bits;
    };

    // One group of 64 steps (four chunks) per iteration, in a fixed order of
    // memory operations: per chunk [window of the chunk two ahead, publish],
    // then [the direction words of the group: one 16-byte store per lane,
    // 1 KiB per wave] [S of the group after next: 16 loads into the slot just
    // consumed].  The prologue issues S of group 0, the first two windows,
    // then S of group 1.  A window is therefore followed by exactly 3 memory
    // operations when its chunk comes, 20 for the first two chunks of a group
    // (17 and 18 in the first group), which is the vmcnt it waits for; a
    // group's S was issued before the window of its first chunk, so that
    // wait also covers the ring.  Without windows (first strip) the ring's
    // own wait is 16, then 21 operations.  A drained counter (after a
    // reload) only makes a wait shorter.  A last group of fewer than four
    // chunks stops after its last chunk; nothing waits after it but the
    // final drain.
    static_assert(RING_GROUPS == 2 && GROUP == 64, "wait counts below assume two ring groups of 64 steps");
    load_group(ring, src, 0, 0);
    if (in_global) {
      prefetch_window(0, winbufA);
      prefetch_window(16, winbufB);
    }
    load_group(ring, src, 1, 1);
    auto take_window = [&](int tw, const uint64_t *buf, int ahead) -> uint64_t {
      // ahead: memory operations issued after this window's load
      if (ahead == 3) asm volatile("s_waitcnt vmcnt(3)" ::: "memory");
      else if (ahead == 20) asm volatile("s_waitcnt vmcnt(20)" ::: "memory");
      else if (ahead == 17) asm volatile("s_waitcnt vmcnt(17)" ::: "memory");
      else asm volatile("s_waitcnt vmcnt(18)" ::: "memory");
      uint64_t v = buf[wslot];
      if (!window_ready(v, tw)) v = wait_window(tw, v);
      return v;
    };
    const int n_groups = src.n_groups;
    int slot = 0;   // ring slot of group q
    for (int q = 0; q < n_groups; ++q) {
      const float *grp = ring + slot * GROUP_FLOATS;
      if (!in_global) {   // the ring slot of group q has landed
        if (q == 0) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
        else asm volatile("s_waitcnt vmcnt(21)" ::: "memory");
      }
      uint32_t bits[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t0 = GROUP * q + 16 * i;
        if (t0 >= T_pad) break;
        uint64_t win = 0ull;
        uint64_t *wbuf = (i & 1) ? winbufB : winbufA;
        if (in_global) {
          win = take_window(t0, wbuf, q == 0 ? (i == 0 ? 17 : i == 1 ? 18 : 3) : (i < 2 ? 20 : 3));
          __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the slot is read before it is refilled
          prefetch_window(t0 + 32, wbuf);
        } else if (link_up) {
          win = link_take(t0);
        }
        if (failed) break;
        bits[i] = chunk(t0, win, grp, off[i]);
      }
      if (failed) break;
      tbs[q * 64 + lane] = make_uint4(bits[0], bits[1], bits[2], bits[3]);
      // every ring read of this group has returned (lgkmcnt(0)) before its
      // slot is refilled with the group after next
      __builtin_amdgcn_s_waitcnt(0xc07f);
      load_group(ring, src, q + RING_GROUPS, slot);
      slot ^= 1;
    }
    // no LDS-direct load may still be writing LDS when the next item starts
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (last) {
      // lane r_last stopped updating after column m: it holds H[n][m]
      const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(st.H), r_last));
      if (lane == 0) score[b] = failed ? __builtin_nanf("") : v;
    } else if (failed) {
      // the strip below must not wait for a row that will never come
      if (link_down) {
        if (lane == 0) __hip_atomic_store(&ctr[wave], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        for (int j = 1 + lane; j <= m; j += 64)
          __hip_atomic_store(out_row + j, (uint64_t)TAG_FAIL << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (failed && lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hot) __builtin_amdgcn_s_setprio(0);
  }
}

// ---- the fill with S staged in registers -----------------------------------------
// The same strip sweep, the same cells, hand-off and publication as k_nw_fill,
// with every memory access an ordinary compiler-tracked load or store: no LDS
// ring and no hand-counted waits.  Lane r loads the 16 cells of its row that
// a 16-step chunk uses (four 16-byte buffer loads of consecutive columns: the
// cell of step t is (r, t - r), byte 4 (r (m - 1) + t) of the strip) two
// chunks ahead into one of three register sets; lanes 0..15 load that chunk's
// boundary window the same way (agent-coherent 8-byte loads).  A cell outside
// the strip's columns reads another cell of the strip, or 0 past its end (the
// buffer range check): only masked steps see it.  Without the 17 KiB ring a
// wave needs registers only, so more waves fit on a compute unit.
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ void load_s16(float4 (&d)[4], __amdgpu_buffer_rsrc_t rs, uint32_t off) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const u32x4v v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u * q, 0, 0);
    d[q] = make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
  }
}

template <bool MAX3>
__global__ __launch_bounds__(64) void k_nw_fill_r(FillArgs A, const float *__restrict__ S, float g,
                                                  float *__restrict__ score, char *__restrict__ tb,
                                                  uint64_t *__restrict__ bnd, int32_t *__restrict__ head,
                                                  int32_t *__restrict__ err) {
  constexpr uint32_t epoch = 1u;   // tag of a published value (the reset clears to 0)
  const int lane = threadIdx.x;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(head, 1);
    item = uniform(item);
    if (item >= A.n_items) break;
    item += A.item0;
    const int b = uniform(A.it_pair[item]);
    const int s_tag = uniform(A.it_strip[item]);
    const int s = s_tag & ~ITEM_HOT;
    const bool hot = (s_tag & ITEM_HOT) != 0;
    if (hot) __builtin_amdgcn_s_setprio(2);
    const int n = uniform(A.n[b]), m = uniform(A.m[b]);
    const int nstrips = (n + 63) >> 6;
    const bool last = s == nstrips - 1;
    const int i0 = 64 * s;
    const int rows = min(64, n - i0);
    const float *Sb = S + A.s_off[b];
    const int64_t mstride = bnd_stride(m);
    const uint64_t *in_row = bnd + A.bnd_off[b] + (int64_t)(s - 1) * mstride;   // used when s > 0
    uint64_t *out_row = bnd + A.bnd_off[b] + (int64_t)s * mstride;               // used when !last
    const int nG = (m + 63 + 63) >> 6;
    uint32_t *tbw = reinterpret_cast<uint32_t *>(reinterpret_cast<uint4 *>(tb + A.tb_off[b]) + (int64_t)s * nG * 64);
    const int T_end = m + rows - 1;
    const int T_pad = (T_end + 15) & ~15;
    const int r_last = n - 1 - i0;   // lane of row n in the last strip
    bool failed = false;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)uniform_ptr(Sb + (int64_t)i0 * m), (short)0, uniform(rows * m * 4), 0x00020000);
    const uint32_t lo = (uint32_t)lane * (uint32_t)(m - 1) * 4u;
    const __amdgpu_buffer_rsrc_t pub_rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)uniform_ptr(out_row), (short)0, last ? 0 : uniform((m + 1) * 8), 0x00020000);

    StripState st;
    const int i = i0 + 1 + lane;
    st.H = (float)i * g;                                    // H[i][0]
    st.diag = (i0 == 0) ? 0.0f : (float)i0 * g;             // lane 0: H[i0][0]
    st.col = 0.0f;
    st.bits = 0u;
    st.pw = 0.0f;

    // the row above: lanes 0..15 hold slots tw + 1 .. tw + 16 (see k_nw_fill)
    auto wload = [&](int tw) -> uint64_t {
      return (s > 0 && lane < 16)
                 ? __hip_atomic_load(in_row + tw + 1 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                 : 0ull;
    };
    auto window_need = [&](int tw) -> bool { return lane < 16 && tw + 1 + lane <= m; };
    auto wait_window = [&](int tw, uint64_t v) -> uint64_t {
      int spins = 0;
      for (;;) {
        const uint32_t tag = (uint32_t)(v >> 32);
        if (__ballot(window_need(tw) && tag == TAG_FAIL) != 0) {
          failed = true;
          break;
        }
        if (__ballot(window_need(tw) && tag != epoch) == 0) break;
        if (++spins > A.spin_limit) {
          failed = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = wload(tw);
      }
      return v;
    };

    float4 SA[4], SB[4], SC[4];
    load_s16(SA, rs, lo);
    uint64_t WA = wload(0);
    load_s16(SB, rs, lo + 64u);
    uint64_t WB = wload(16), WC = 0ull;
    int t0 = 0;
    // one 16-step chunk from register set CUR while chunk t0 + 32 loads into NXT
#define NWM_FILL_RCHUNK(CUR, WCUR, NXT, WNXT)                                                       \
  {                                                                                                \
    if (t0 >= T_pad) break;                                                                        \
    load_s16(NXT, rs, lo + 4u * (uint32_t)(t0 + 32));                                              \
    WNXT = wload(t0 + 32);                                                                         \
    uint64_t win = WCUR;                                                                           \
    if (s > 0 && __ballot(window_need(t0) && (uint32_t)(win >> 32) != epoch) != 0) {               \
      win = wait_window(t0, win);                                                                  \
      if (failed) break;                                                                           \
    }                                                                                              \
    st.pw = s > 0 ? __uint_as_float((uint32_t)win) : (float)(t0 + 1 + lane) * g;                  \
    if (t0 < 64 || t0 + 16 > m) run16v<true, MAX3>(st, CUR, t0, m, g, lane);                      \
    else run16v<false, MAX3>(st, CUR, t0, m, g, lane);                                             \
    {                                                                                              \
      const int j = t0 - 110 + lane;                                                               \
      const bool pub = !last && lane >= 48 && j >= 1 && j <= m && !(A.hold && s == 0);             \
      publish(pub_rs, pub, j, ((uint64_t)epoch << 32) | __float_as_uint(st.col));                  \
    }                                                                                              \
    tbw[((t0 >> 6) * 64 + lane) * 4 + ((t0 >> 4) & 3)] = st.bits;                                  \
    t0 += 16;                                                                                      \
  }
    for (;;) {
      NWM_FILL_RCHUNK(SA, WA, SC, WC)
      NWM_FILL_RCHUNK(SB, WB, SA, WA)
      NWM_FILL_RCHUNK(SC, WC, SB, WB)
    }
#undef NWM_FILL_RCHUNK
    if (last) {
      // lane r_last stopped updating after column m: it holds H[n][m]
      const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(st.H), r_last));
      if (lane == 0) score[b] = failed ? __builtin_nanf("") : v;
    } else if (failed) {
      for (int j = 1 + lane; j <= m; j += 64)
        __hip_atomic_store(out_row + j, (uint64_t)TAG_FAIL << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (failed && lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hot) __builtin_amdgcn_s_setprio(0);
  }
}

constexpr int WALK_LDS = 2048;   // path cells buffered in LDS per pair before a flush

// One 1 KiB block of direction words into LDS (lane l: bytes 16 l .. 16 l +
// 15 of blk), LDS-direct so that no register is written while the load is in
// flight (the compiler takes an asm load's outputs as written at issue and
// may copy them).  Readers wait with an explicit vmcnt.
static __device__ __forceinline__ void load_block_lds(uint4 *blk, const uint4 *src) {
  const uint32_t la = (uint32_t)uniform((int)(uint32_t)(uintptr_t)(lds_void *)blk);
  uint32_t save;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(save)
      : "s"(la), "v"(src)
      : "memory");
}

// The 2-bit code at position p (0..63) of a block row held as four words of
// 16 codes (first position in the high bits); w0..w3 may be per lane.
static __device__ __forceinline__ uint32_t code_at(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, int p) {
  const int q = p >> 4;
  const uint32_t w = q == 0 ? w0 : q == 1 ? w1 : q == 2 ? w2 : w3;
  return (w >> (2 * (15 - (p & 15)))) & 3u;
}

// The 16 flags at even bit positions 2 m of x (bits 2 m + 1 ignored) packed
// into bits m.
static __device__ __forceinline__ uint32_t pack_even(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  return (x | (x >> 8)) & 0x0000FFFFu;
}

// Traceback (Sec. 5.1): from (n, m) back to the first row or column,
// following the stored directions; every DIAG step emits the aligned pair.
// One wave per pair (longest pair first).  Position: strip s, row r of the
// strip (lane r), anti-diagonal step t = j - 1 + r; the walk holds the 1 KiB
// block of codes covering steps [64 G, 64 G + 64) of the strip (lane l: row
// l's four words), and each lane turns its row into two 64-bit masks, bit
// 63 - p for step 64 G + p: codes other than LEFT, and DIAG codes.  The walk
// then moves by runs: from step t of row r the path goes LEFT up to the
// first code that is not LEFT at or before t (the lowest set bit of the
// row's mask above bit 63 - (t - 64 G), found on the scalar unit) and leaves
// the row there by DIAG (step - 2) or UP (step - 1); every lane below tests
// its row's code where that move enters it, and a ballot finds the first row
// where the run of the same move ends, so a LEFT run and the DIAG or UP run
// after it are one iteration.  The DIAG cells are recorded per lane (one per
// row and strip) and written to LDS together, in path order, when the walk
// leaves the strip.  The walk is bound by the latency
// of its steps, and of its block loads, so each strip's blocks are
// requested a whole strip ahead: the wave holds four blocks of its strip in
// LDS and, on entering a strip, requests the four blocks of the strip above
// that the path will cross if it keeps the pair's average slope (m / n
// columns per row; within a strip the step only decreases, by one block at
// a time).  A block outside those four is loaded when it is reached, and
// from then on the block to its left is prefetched.  Path cells reach memory
// in coalesced stores.
__global__ __launch_bounds__(64) void k_nw_walk(PlanDev P, const char *__restrict__ tb_bits,
                                                const float *__restrict__ score, int2 *__restrict__ path,
                                                int32_t *__restrict__ n_diag, int o0) {
  __shared__ int2 lbuf[WALK_LDS];
  // two sets of four blocks (slots 4 k .. 4 k + 3), then the block on the left
  __shared__ uint4 wblk[9 * 64];
  const int b = P.dp_order[o0 + blockIdx.x];
  const int n = P.n[b], m = P.m[b];
  const int lane = threadIdx.x;
  const int cap = min(n, m);
  int2 *pa = path + P.p_off[b];   // entry q of the walk (descending) at cap - 1 - q
  // an empty side, or a fill that gave up (NaN score): no aligned pairs
  if (n <= 0 || m <= 0 || __builtin_isnan(score[b])) {
    if (lane == 0) n_diag[b] = 0;
    return;
  }
  const uint4 *tbw = reinterpret_cast<const uint4 *>(tb_bits + P.tb_off[b]);
  const int nS = (n + 63) >> 6;
  const int nG = (m + 63 + 63) >> 6;
  auto blk_ptr = [&](int s, int G) {
    // out-of-range candidates read block (0, 0), which always exists
    const bool ok = s >= 0 && s < nS && G >= 0 && G < nG;
    return tbw + (ok ? ((int64_t)s * nG + G) * 64 : 0) + lane;
  };
  // position: strip s, row r, step t  (i = 64 s + r + 1, j = t - r + 1)
  int s = (n - 1) >> 6, r = (n - 1) & 63, t = m - 1 + r;
  int k = 0, kb = 0, flushed = 0;   // cells emitted; cells in lbuf; cells stored
  // set hs holds blocks ob .. ob + 3 of strip cs; the other set blocks
  // ab .. ab + 3 of strip cs - 1 (in flight until the strip changes); slot 8
  // block cG - 1 of strip cs, in flight while pa_live
  int cs = s, cG = t >> 6;
  // the entry step of the strip above, relative to this strip's, for a path
  // of the average slope: one row up (+64 steps) after 64 rows of slope m / n
  const int d = 1 - (int)(((int64_t)64 * m) / n);
  auto load_slot = [&](int slot, int bs, int bG) { load_block_lds(&wblk[slot * 64], blk_ptr(bs, bG)); };
  // the four blocks ending with the one 32 steps right of the predicted entry
  auto above_base = [&](int t_in) { return ((t_in + d + 32) >> 6) - 3; };
  int hs = 0, ob = cG - 3, ab = above_base(t);
  for (int q = 0; q < 4; ++q) load_slot(q, cs, ob + q);
  for (int q = 0; q < 4; ++q) load_slot(4 + q, cs - 1, ab + q);
  asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  auto flush = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < kb; e += 64) {
      const int q = flushed + e;
      if (q < cap) pa[cap - 1 - q] = lbuf[e];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    flushed += kb;
    kb = 0;
  };
  bool pa_live = false;
  // this lane's row of the current block as masks (bit 63 - p: step 64 G + p):
  // codes other than LEFT, DIAG codes, the other codes (UP)
  uint64_t nl = 0ull, dg = 0ull, up = 0ull;
  auto row_masks = [&](const uint4 &w) {
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
    nl = 0ull;
    dg = 0ull;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // code at position k of word q in bits 2 (15 - k) + 1 .. 2 (15 - k):
      // DIAG 0, UP 1, LEFT 2
      const uint32_t hi = ws[q] >> 1, lo = ws[q];
      nl |= (uint64_t)pack_even(~hi | lo) << (16 * (3 - q));
      dg |= (uint64_t)pack_even(~(hi | lo)) << (16 * (3 - q));
    }
    up = nl & ~dg;
  };
  row_masks(wblk[3 * 64 + lane]);
  int cell = -1;   // this lane's row: the step of its DIAG cell in the current strip
  // the current strip's DIAG cells to LDS, rows in descending order
  auto emit = [&]() {
    const uint64_t has = __ballot(cell >= 0);
    if (has == 0ull) return;
    const int nc = __popcll(has);
    if (kb + nc > WALK_LDS) flush();
    if (cell >= 0) lbuf[kb + __popcll(lane == 63 ? 0ull : has >> (lane + 1))] = make_int2(64 * s + lane, cell - lane);
    kb += nc;
    k += nc;
    cell = -1;
  };
  for (;;) {
    if (r < 0) {   // into the strip above
      emit();
      --s;
      r += 64;
      t += 64;
    }
    if (s < 0 || t - r < 0) break;   // i == 0 or j == 0
    const int G = t >> 6;
    if (s != cs) {
      // into the strip above (s = cs - 1): its blocks, requested a strip
      // ago, become the held set, and the set just left (read for the last
      // time at an earlier block change) takes the strip above this one
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      hs ^= 1;
      ob = ab;
      cs = s;
      cG = G + 1;   // select below
      pa_live = false;
      ab = above_base(t);
      for (int q = 0; q < 4; ++q) load_slot(4 * (hs ^ 1) + q, cs - 1, ab + q);
    }
    if (G != cG) {
      // within a strip the walk only moves to the block on the left
      const int x = G - ob;
      int slot = 8;
      if (x >= 0 && x < 4) {
        slot = 4 * hs + x;
      } else if (pa_live && G == cG - 1) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      } else {
        load_slot(8, s, G);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      }
      row_masks(wblk[slot * 64 + lane]);
      pa_live = false;
      cG = G;
      if (G - 1 < ob && G >= 1) {   // past the held blocks: prefetch the next one to the left
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): slot 8 has been read before it is refilled
        load_slot(8, s, G - 1);
        pa_live = true;
      }
    }
    const int base = 64 * G;
    const uint64_t nlr = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(nl >> 32), r) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)nl, r);
    const uint64_t dgr = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dg >> 32), r) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)dg, r);
    const uint64_t x = nlr & (~0ull << (63 - (t - base)));
    if (x == 0ull) {   // LEFT past the block's first step: on in block G - 1
      t = base - 1;
      continue;
    }
    const int bb = __builtin_ctzll(x);
    const int tp = base + 63 - bb;   // the step where the path leaves row r
    if (tp < r) break;               // the LEFT run reaches column 0 first
    const bool diag = (dgr >> bb) & 1ull;
    // the run of DIAG (or UP) moves from tp: row rho < r is entered at step
    // tp - slope (r - rho) and continues the run if its code there is the
    // same; the first row (from r down) where it is not, or where the step
    // leaves the block or column 1, is where the next iteration starts
    const int slope = diag ? 2 : 1;
    const int tq = tp - slope * (r - lane);
    const int pq = tq - base;
    const uint64_t same = diag ? dg : up;
    const bool ok = lane < r && pq >= 0 && tq >= lane && ((same >> ((63 - pq) & 63)) & 1ull);
    const uint64_t brk = __ballot(!ok) & ((1ull << r) - 1ull);
    const int rs = brk ? 63 - __builtin_clzll(brk) : -1;   // highest breaking row below r
    if (diag && lane > rs && lane <= r) cell = tq;
    t = tp - slope * (r - rs);
    r = rs;
  }
  emit();
  // no LDS-direct load may still be writing LDS when the wave ends
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  flush();
  if (lane == 0) n_diag[b] = k;
}

__global__ __launch_bounds__(64) void k_keep(PlanDev P, const float *__restrict__ S, float thr,
                                             const int2 *__restrict__ path, const int32_t *__restrict__ n_diag,
                                             int2 *__restrict__ kept, int32_t *__restrict__ n_kept, int o0) {
  const int b = P.dp_order[o0 + blockIdx.x];
  const int n = P.n[b], m = P.m[b];
  const int lane = threadIdx.x;
  const int cap = min(n, m);
  const int k = min(n_diag[b], cap);
  const int2 *pa = path + P.p_off[b] + (cap - k);
  int2 *kp = kept + P.p_off[b];
  const float *Sb = S + P.s_off[b];
  int nk = 0;
  // 256 path cells per round: the four path loads, then the four S loads
  // that depend on them, are each in flight together
  constexpr int U = 4;
  for (int q0 = 0; q0 < k; q0 += 64 * U) {
    int2 c[U];
    float sv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + 64 * u + lane;
      c[u] = q < k ? pa[q] : make_int2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + 64 * u + lane;
      sv[u] = q < k ? Sb[(int64_t)c[u].x * m + c[u].y] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool keep = q0 + 64 * u + lane < k && sv[u] >= thr;
      const uint64_t km = __ballot(keep);
      if (keep) kp[nk + __popcll(km & ((1ull << lane) - 1ull))] = c[u];
      nk += __popcll(km);
    }
  }
  if (lane == 0) n_kept[b] = nk;
}

// compute units; resident fill workgroups per unit for the LDS-ring fill
// with tasks of FILL_SLOTS strips and with single strips, and resident waves
// for the register staging
static int g_fill_cus = 0, g_fill_per = 0, g_fill_per1 = 0, g_fill_per_r = 0;

template <int SLOTS>
static hipError_t fill_ring_attrs(int &per) {
  int a = 0, c = 0;
  hipError_t e = hipFuncSetAttribute((const void *)k_nw_fill<false, SLOTS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     fill_lds_bytes(SLOTS));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_nw_fill<true, SLOTS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            fill_lds_bytes(SLOTS));
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_nw_fill<false, SLOTS>, 64 * SLOTS, fill_lds_bytes(SLOTS));
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_nw_fill<true, SLOTS>, 64 * SLOTS, fill_lds_bytes(SLOTS));
  per = a < c ? a : c;   // either variant's grid is resident at once
  if (per < 1) per = 1;
  return e;
}

hipError_t fill_set_attrs(int) {
  if (g_fill_cus == 0) {
    int dev = 0, cus = 0, per = 0, per1 = 0, pr = 0, pr3 = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the four-strip fill takes more than the default 64 KiB of LDS per workgroup
    if (e == hipSuccess) e = fill_ring_attrs<FILL_SLOTS>(per);
    if (e == hipSuccess) e = fill_ring_attrs<1>(per1);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pr, k_nw_fill_r<false>, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pr3, k_nw_fill_r<true>, 64, 0);
    if (e != hipSuccess) return e;
    pr = pr < pr3 ? pr : pr3;   // either variant's grid is resident at once
    g_fill_per = per;
    g_fill_per1 = per1;
    g_fill_per_r = pr > 0 ? pr : 1;
    g_fill_cus = cus > 0 ? cus : 1;
  }
  return hipSuccess;
}

static FillArgs fill_args(const PlanDev &P) {
  FillArgs A;
  A.n_items = P.n_items;
  A.B = P.B;
  A.item0 = 0;
  A.n_tasks = P.n_tasks;
  A.task0 = 0;
  A.spin_limit = SPIN_LIMIT;
  A.hold = 0;
  A.it_pair = P.it_pair;
  A.it_strip = P.it_strip;
  A.tk_pair = P.tk_pair;
  A.tk_slot = P.tk_slot;
  A.n = P.n;
  A.m = P.m;
  A.s_off = P.s_off;
  A.tb_off = P.tb_off;
  A.bnd_off = P.bnd_off;
  return A;
}

// Clears the published-row region and the queue heads; scores of empty pairs.
hipError_t launch_nw_reset(const PlanDev &P, float g, float *score, uint64_t *bnd, int64_t n_bnd, int32_t *ctl,
                           hipStream_t st) {
  if (P.B <= 0) return hipSuccess;
  const int64_t n16 = (n_bnd + 1) / 2;   // the region is 256-byte aligned and padded
  const int64_t rb = (n16 + 255) / 256;
  hipLaunchKernelGGL(k_nw_reset, dim3((unsigned)(rb < 2048 ? (rb > 0 ? rb : 1) : 2048)), dim3(256), 0, st,
                     fill_args(P), reinterpret_cast<uint4 *>(bnd), n16, ctl, g, score);
  return hipGetLastError();
}

// DP items [item0, item0 + n) of the plan (the register staging) or the same
// strips as tasks [task0, task0 + nt) (the LDS ring), popped from the queue
// head `head` (cleared by the reset).  Strips of one pair must all be in one
// launch.
hipError_t launch_nw_fill_items(const PlanDev &P, const float *S, float g, float *score, char *tb, uint64_t *bnd,
                                int64_t n_bnd, int32_t *head, int32_t *err, int item0, int n, int task0, int nt,
                                int waves_per_cu, int spin_limit, int hold, int staging, hipStream_t st) {
  if (P.B <= 0 || n <= 0) return hipSuccess;
  if (g_fill_cus == 0) {
    hipError_t e = fill_set_attrs(0);
    if (e != hipSuccess) return e;
  }
  FillArgs A = fill_args(P);
  A.item0 = item0;
  A.n_items = n;
  A.task0 = task0;
  A.n_tasks = nt;
  A.spin_limit = spin_limit > 0 ? spin_limit : SPIN_LIMIT;
  A.hold = hold;
  // every wave of the grid is resident at once (the hand-off between strips
  // waits on other waves), so the grid never exceeds the occupancy; for the
  // LDS ring, waves_per_cu counts the waves of whole workgroups.  Staging 0:
  // LDS ring, tasks of FILL_SLOTS strips; 2: LDS ring, one strip per
  // workgroup (the plan's items as tasks of one); 1: registers.
  const bool max3 = !(g == 0.0f && std::signbit(g));   // a gap of -0 keeps the compare chain (see run16v)
  if (staging == 1) {
    const int per = (waves_per_cu > 0 && waves_per_cu < g_fill_per_r) ? waves_per_cu : g_fill_per_r;
    const int grid = std::min(n, g_fill_cus * per);
    if (max3)
      hipLaunchKernelGGL(k_nw_fill_r<true>, dim3(grid), dim3(64), 0, st, A, S, g, score, tb, bnd, head, err);
    else
      hipLaunchKernelGGL(k_nw_fill_r<false>, dim3(grid), dim3(64), 0, st, A, S, g, score, tb, bnd, head, err);
  } else if (staging == 2) {
    A.tk_pair = P.it_pair;
    A.tk_slot = P.it_strip;
    A.task0 = item0;
    A.n_tasks = n;
    int per = g_fill_per1;
    if (waves_per_cu > 0 && waves_per_cu < per) per = waves_per_cu;
    const int grid = std::min(n, g_fill_cus * per);
    constexpr int lds = fill_lds_bytes(1);
    if (max3)
      hipLaunchKernelGGL((k_nw_fill<true, 1>), dim3(grid), dim3(64), lds, st, A, S, g, score, tb, bnd, head, err);
    else
      hipLaunchKernelGGL((k_nw_fill<false, 1>), dim3(grid), dim3(64), lds, st, A, S, g, score, tb, bnd, head, err);
  } else {
    int groups = g_fill_cus * g_fill_per;
    if (waves_per_cu > 0) groups = std::min(groups, std::max(1, g_fill_cus * waves_per_cu / FILL_SLOTS));
    const int grid = std::min(nt, groups);
    constexpr int lds = fill_lds_bytes(FILL_SLOTS);
    if (max3)
      hipLaunchKernelGGL((k_nw_fill<true, FILL_SLOTS>), dim3(grid), dim3(64 * FILL_SLOTS), lds, st, A, S, g, score, tb,
                         bnd, head, err);
    else
      hipLaunchKernelGGL((k_nw_fill<false, FILL_SLOTS>), dim3(grid), dim3(64 * FILL_SLOTS), lds, st, A, S, g, score,
                         tb, bnd, head, err);
  }
  return hipGetLastError();
}

hipError_t launch_nw_fill(const PlanDev &P, const float *S, float g, float *score, char *tb, uint64_t *bnd,
                          int64_t n_bnd, int32_t *ctl, int waves_per_cu, int spin_limit, int hold, int staging,
                          hipStream_t st) {
  hipError_t e = launch_nw_reset(P, g, score, bnd, n_bnd, ctl, st);
  if (e != hipSuccess) return e;
  return launch_nw_fill_items(P, S, g, score, tb, bnd, n_bnd, ctl, ctl + 1, 0, P.n_items, 0, P.n_tasks, waves_per_cu,
                              spin_limit, hold, staging, st);
}

// pairs dp_order[o0 .. o0 + n)
hipError_t launch_nw_walk(const PlanDev &P, const char *tb, const float *score, int2 *path, int32_t *n_diag, int o0,
                          int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nw_walk, dim3(n), dim3(64), 0, st, P, tb, score, path, n_diag, o0);
  return hipGetLastError();
}

hipError_t launch_keep(const PlanDev &P, const float *S, float thr, const int2 *path, const int32_t *n_diag,
                       int2 *kept, int32_t *n_kept, int o0, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keep, dim3(n), dim3(64), 0, st, P, S, thr, path, n_diag, kept, n_kept, o0);
  return hipGetLastError();
}

}  // namespace nwm
