// Device kernels of tsmg for gfx950 (CDNA4, wave64).
//
// Hot path (per operator apply A_g c, Sec. 2.4 / Alg. 2-4 of arXiv:1901.00654):
//   k_lambda_fused2/3, k_lambda_pass
//                  out  = lambda Lambda_g c (one kernel for d = 2, 3; for
//                  d >= 4 one banded pass per leading dimension, then the
//                  d = 3 kernel over the last three dimensions)
//   k_data<kApply> out += Phi_g'(Phi_g c), points sorted by knot cell,
//                  segments and items from a work list built on the host,
//                  coefficient patch of a cell tile staged in LDS, per-point
//                  tensor basis as products of 1D cubic values in registers,
//                  scatter reduced in LDS before one atomic per patch entry.
//   k_stencil_apply(_small)
//                  out = A_g x on levels assembled as 7^d-point stencils
//                  (half stored, A_g being symmetric), with Jacobi /
//                  residual epilogues.
// V-cycle pieces: Jacobi kernels (Alg. 6), subdivision prolongation and
// restriction, pass by pass or fused (Sec. 3.2.3), coarse GEMV with the
// precomputed inverse (Sec. 3.2.4); CG vector kernels with device-resident
// scalars (Alg. 8).
// Setup: binning, offsets, Jacobi diagonal (Alg. 5 + Kronecker diagonal),
// stencil assembly from per-cell polynomial moments (read from the points
// on the finest assembled level, carried to coarser ones by a change of
// variables), Gauss-Jordan inversion of A_1.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace tsmg {

// ---------------------------------------------------------------------------
// Cubic uniform B-spline pieces on one knot interval, t in [0,1]: the four
// functions alive there (indices c..c+3 of the cell c), written out from the
// de Boor recursion on uniform knots.
template <typename T>
__device__ __forceinline__ void cubic_basis(T t, T (&b)[4]) {
  const T s = T(1) - t;
  const T t2 = t * t, s2 = s * s;
  const T t3 = t2 * t, s3 = s2 * s;
  const T sixth = T(1.0 / 6.0), two3 = T(2.0 / 3.0), half = T(0.5);
  b[0] = s3 * sixth;
  b[1] = two3 - t2 + half * t3;
  b[2] = two3 - s2 + half * s3;
  b[3] = t3 * sixth;
}

// Morton (bit-interleaved) index -> per-dimension coordinates, `bits` bits
// per dimension, dimension 0 most significant inside each bit group.
template <int D>
__device__ __forceinline__ void morton_decode(uint32_t key, int bits, int (&c)[D]) {
#pragma unroll
  for (int p = 0; p < D; ++p) c[p] = 0;
  for (int b = 0; b < bits; ++b) {
#pragma unroll
    for (int p = 0; p < D; ++p) c[p] |= int((key >> (b * D + (D - 1 - p))) & 1u) << b;
  }
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// blockIdx. This renumbering gives each XCD a contiguous run of logical
// blocks, so neighbouring point ranges - which share tiles, coefficient
// patches and output entries - run behind the same L2. It is a bijection of
// 0..gridDim.x-1.
__device__ __forceinline__ int xcd_block() {
  constexpr int kXcd = 8;
  const int nb = gridDim.x, b = blockIdx.x;
  const int x = b % kXcd, q = nb / kXcd, r = nb % kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// ---------------------------------------------------------------------------
// Unrolled, sum-factorised tensor-product gather over the innermost
// dimensions p..D-1 of a patch with strides st[] (last stride 1), innermost
// 4-term rows first (used by the evaluation of a fit).
template <int D, int p, typename T>
struct Inner {
  static __device__ __forceinline__ T gather(const T* lc, int o, const T (&B)[D][4],
                                             const int (&st)[D]) {
    T r = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) r += B[p][a] * Inner<D, p + 1, T>::gather(lc, o + a * st[p], B, st);
    return r;
  }
};
template <int D, typename T>
struct Inner<D, D, T> {
  static __device__ __forceinline__ T gather(const T* lc, int o, const T (&)[D][4], const int (&)[D]) {
    return lc[o];
  }
};

// Dimensions 1..D-1 are unrolled at compile time for D = 5 and dimension 0
// runs as a 4-step loop that rotates its four basis values through fixed
// registers, so no array is ever indexed at run time (which would put the
// basis values in scratch memory). For D <= 4 everything is unrolled.
template <int D>
struct Split {
  static constexpr int L = (D <= 4) ? 0 : 1;
};

template <int D, typename T>
__device__ __forceinline__ T patch_gather(const T* lc, int base, const T (&B)[D][4], const int (&st)[D]) {
  if constexpr (Split<D>::L == 0) {
    return Inner<D, 0, T>::gather(lc, base, B, st);
  } else {
    T s = T(0);
    T r0 = B[0][0], r1 = B[0][1], r2 = B[0][2], r3 = B[0][3];
    int o = base;
#pragma unroll 1
    for (int a = 0; a < 4; ++a) {
      s += r0 * Inner<D, 1, T>::gather(lc, o, B, st);
      r0 = r1; r1 = r2; r2 = r3;
      o += st[0];
    }
    return s;
  }
}

// ---------------------------------------------------------------------------
// The data term of one level: out += Phi_g'(Phi_g c) (kApply), Phi_g'y (kRhs)
// or diag(Phi_g'Phi_g) (kDiag).
//
// Work split. Workgroup w owns the sorted points [w*ppb, (w+1)*ppb). Points
// are in Morton order of their finest cell, so each Morton-aligned tile of
// 2^tb level-g cells per dimension is one contiguous point range. Per tile
// segment the workgroup stages the (2^tb + 3)^D coefficient patch in LDS and
// cuts the segment into items: runs of at most Q points of one cell (read
// from the level's work list, or derived from the cell offsets on the fly).
//
// Items go to lane groups of L = 4^(D-2) lanes (one lane for D <= 2; eight
// for D = 3). A lane holds 16 coefficients of the cell's 4^D patch in
// registers - the last two dimensions, for its own fixed leading
// multi-index - and 16 accumulators (at D = 3 eight of each: its half of
// dimension 1, which leaves registers for six waves per SIMD instead of
// four: 77 against 83 us at C2). Per point the group evaluates the cubic pieces (the lane's
// own factor of the leading dimensions by Horner, the four values of each
// of the last two dimensions), gathers s = v'c (sum-factorised, then summed
// over the group by shuffles) and scatters s v into its accumulators. After
// the item, the accumulators are added into the tile's LDS accumulator, and
// after the tile, the LDS accumulator is added to the output with one
// global atomic per nonzero entry.
// Exclusive prefix sum over the workgroup (one value per thread); *total gets
// the sum. Contains __syncthreads: every thread must call it.
__device__ __forceinline__ int block_exclusive_scan(int v, int* wave_sums, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wave_sums[wid] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const int sw = wave_sums[w];
    before += (w < wid) ? sw : 0;
    tot += sw;
  }
  __syncthreads();
  *total = tot;
  return before + x - v;
}

constexpr int kMaxTileCells = 256;   // cells of one tile, at most (one per thread)

template <int D>
struct Group {
  static constexpr int L = (D <= 2) ? 1 : (D == 3 ? 8 : (1 << (2 * (D - 2))));   // lanes per item
  static constexpr int V = (D == 1) ? 4 : (D == 3 ? 8 : 16);                      // coefficients per lane
  static constexpr int Q = kItemQ[D];                              // points per item
  static constexpr int NG = kBlock / L;                            // groups per workgroup
  static constexpr int PPB = kMaxPointsPerBlock[D];                // points per workgroup, at most
  static constexpr int MAXI = PPB / Q + kMaxTileCells;             // items per tile segment, at most
  static constexpr bool STAGE_C = D <= 4;                          // coefficient patch in LDS
};

// Polynomial coefficients (t^0..t^3) of the cubic piece b_a on one interval.
template <typename T>
__device__ __forceinline__ void piece_coeffs(int a, T& c0, T& c1, T& c2, T& c3) {
  if (a == 0) { c0 = T(1.0 / 6.0); c1 = T(-0.5); c2 = T(0.5); c3 = T(-1.0 / 6.0); }
  else if (a == 1) { c0 = T(2.0 / 3.0); c1 = T(0.0); c2 = T(-1.0); c3 = T(0.5); }
  else if (a == 2) { c0 = T(1.0 / 6.0); c1 = T(0.5); c2 = T(0.5); c3 = T(-0.5); }
  else { c0 = T(0.0); c1 = T(0.0); c2 = T(0.0); c3 = T(1.0 / 6.0); }
}

// Cross-lane moves inside a quad / a row of 16 lanes (DPP, no LDS round trip).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRowRor4 = 0x124;   // row_ror:4
constexpr int kDppRowRor8 = 0x128;   // row_ror:8

// Sum over the L consecutive lanes of a group (L = 1, 4, 16 or 64); every
// lane of the group gets the total.
template <typename T, int L>
__device__ __forceinline__ T group_sum(T v) {
  if constexpr (L >= 4) {
    v += dpp_mov<kDppQuadXor1>(v);
    v += dpp_mov<kDppQuadXor2>(v);
  }
  if constexpr (L == 8) v += dpp_mov<0x141>(v);   // row_half_mirror: the other quad of the eight
  if constexpr (L >= 16) {
    v += dpp_mov<kDppRowRor4>(v);
    v += dpp_mov<kDppRowRor8>(v);
  }
  if constexpr (L >= 64) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
  }
  return v;
}

// Per-point values of one lane: its factor of the leading dimensions (w) and
// the four cubic values of the last two dimensions (bm2, bm1).
template <int D, typename T>
struct PointVals {
  T w;
  T bm1[4];
  T bm2[4];
};

template <int D, typename T, int NLEAD>
__device__ __forceinline__ void point_basis(const T* s_tt, int ppb, int li, const T (&hc)[NLEAD > 0 ? NLEAD : 1][4],
                                            PointVals<D, T>& q) {
  T tt[D];
#pragma unroll
  for (int p = 0; p < D; ++p) tt[p] = s_tt[p * ppb + li];
  q.w = T(1);
#pragma unroll
  for (int k = 0; k < NLEAD; ++k) q.w *= ((hc[k][3] * tt[k] + hc[k][2]) * tt[k] + hc[k][1]) * tt[k] + hc[k][0];
  cubic_basis(tt[D - 1], q.bm1);
  if constexpr (D >= 2) cubic_basis(tt[D - 2], q.bm2);
}

// The lane's share of v'c (before the factor w): sum over its 16 (or 4) entries.
template <int D, typename T, int V>
__device__ __forceinline__ T point_gather(const PointVals<D, T>& q, const T (&cv)[V]) {
  T tl = T(0);
  if constexpr (D == 1) {
#pragma unroll
    for (int b = 0; b < 4; ++b) tl += q.bm1[b] * cv[b];
  } else {
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      T r = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) r += q.bm1[b] * cv[aa * 4 + b];
      tl += q.bm2[aa] * r;
    }
  }
  return tl;
}

// acc += s v (or s v.^2 for the diagonal) over the lane's entries.
template <int D, typename T, bool SQ, int V>
__device__ __forceinline__ void point_scatter(const PointVals<D, T>& q, T s, T (&acc)[V]) {
  const T u = SQ ? s * q.w * q.w : s * q.w;
  if constexpr (D == 1) {
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] += SQ ? u * q.bm1[b] * q.bm1[b] : u * q.bm1[b];
  } else {
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      const T ua = SQ ? u * q.bm2[aa] * q.bm2[aa] : u * q.bm2[aa];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[aa * 4 + b] += SQ ? ua * q.bm1[b] * q.bm1[b] : ua * q.bm1[b];
    }
  }
}

// Dynamic LDS of the point pass, in this order: the staged coefficient patch
// (apply with staging), the FP64 patch accumulator, the staged point
// positions [D][ppb], and the segment's items (work list: one packed word per
// item; otherwise cell, first point and count tables).
struct DataLds {
  size_t lacc, tt, items, slots, cells, total;
};
__host__ __device__ constexpr size_t lds_round(size_t b) { return (b + 15) & ~size_t(15); }
__host__ __device__ constexpr int max_items(int ppb, int Q) { return ppb / Q + 256; }

// With DET the per-item accumulators of one round (kBlock x V FP64) and the
// round's item cells (one per lane group) follow.
template <int D, typename T, int MODE, bool STAGE_C, bool WL, bool DET = false>
__host__ __device__ constexpr DataLds data_lds(int patch, int ppb, int Q) {
  DataLds l{};
  l.lacc = (MODE == kApply && STAGE_C) ? lds_round(size_t(patch) * sizeof(T)) : 0;
  l.tt = l.lacc + lds_round(size_t(patch) * sizeof(double));
  l.items = l.tt + lds_round(size_t(D) * size_t(ppb) * sizeof(T));
  l.slots = l.items + lds_round(size_t(max_items(ppb, Q)) * sizeof(int) * (WL ? 1 : 3));
  l.cells = l.slots + (DET ? lds_round(size_t(kBlock) * (D == 1 ? 4 : 16) * sizeof(double)) : 0);
  l.total = l.cells + (DET ? size_t(kBlock) * sizeof(int) : 0);
  return l;
}

// TBF >= 0: the tile side is 2^TBF (known at compile time, the usual case);
// TBF < 0: it is a.tb (levels coarser than one full tile). WL: take the
// segments and items from the level's precomputed work list instead of
// deriving them from the sorted keys and cell offsets. DET (with WL, whose
// segments are single chunks): the run-to-run reproducible form - the items
// of a segment are taken in rounds of one per lane group, each round's
// accumulators are published in LDS and every patch entry adds them in lane
// group order (no LDS atomics), and the segment's patch is stored to
// det_part[chunk] for k_det_reduce instead of being added to the output with
// atomics.
template <int D, typename T, int MODE, int TBF, bool WL, bool DET = false>
__global__ __launch_bounds__(kBlock) void k_data(DataArgs a) {
  using GP = Group<D>;
  constexpr int L = GP::L;
  constexpr int V = GP::V;
  constexpr int Q = GP::Q;
  constexpr int NLEAD = (D >= 3) ? D - 2 : 0;       // dimensions owned by the lane index
  constexpr bool STAGE_C = GP::STAGE_C;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int scan_sh[kBlock / 64];

  T* lc = reinterpret_cast<T*>(smem_raw);
  const int tbits = TBF >= 0 ? TBF : a.tb;
  const int Tg = 1 << tbits;
  const int P = Tg + kDeg;
  int patch = 1;
#pragma unroll
  for (int p = 0; p < D; ++p) patch *= P;
  // the patch accumulator is FP64 for both precisions: LDS float atomics are
  // several times slower than FP64 ones on gfx950
  static_assert(!DET || WL, "the deterministic form runs from a work list");
  const DataLds lay = data_lds<D, T, MODE, STAGE_C, WL, DET>(patch, a.ppb, Q);
  double* lacc = reinterpret_cast<double*>(smem_raw + lay.lacc);
  T* s_tt = reinterpret_cast<T*>(smem_raw + lay.tt);   // [D][ppb] level-g positions in the cell
  const int maxi = max_items(a.ppb, Q);
  uint32_t* s_items = reinterpret_cast<uint32_t*>(smem_raw + lay.items);
  int* it_cell = reinterpret_cast<int*>(s_items);
  int* it_lo = it_cell + maxi;
  int* it_cnt = it_lo + maxi;
  double* s_slot = reinterpret_cast<double*>(smem_raw + lay.slots);   // DET: [kBlock][V]
  int* s_jcell = reinterpret_cast<int*>(smem_raw + lay.cells);         // DET: [lane groups]

  int st[D];
  st[D - 1] = 1;
#pragma unroll
  for (int p = D - 2; p >= 0; --p) st[p] = st[p + 1] * P;

  const int Jg = (1 << a.g) + kDeg;
  const int sh = a.G - a.g;                       // finest -> level g shift
  const uint32_t maskN = (1u << a.G) - 1u;
  const uint32_t maskSh = (1u << sh) - 1u;
  const T scale = T(1.0) / T(double(1u << sh));   // exact power of two
  const int S = D * (sh + tbits);                  // finest Morton key -> tile index
  const int cells_in_tile = 1 << (D * tbits);
  const T* tfrac = reinterpret_cast<const T*>(a.tfrac);
  const T* cin = reinterpret_cast<const T*>(a.c);
  T* out = reinterpret_cast<T*>(a.out);

  // the lane's place in its group and its fixed leading multi-index
  const int grp = threadIdx.x / L;
  const int lig = threadIdx.x % L;
  T hc[NLEAD > 0 ? NLEAD : 1][4];
  int lead_off = 0;
#pragma unroll
  for (int q = 0; q < NLEAD; ++q) {
    const int aq = (D == 3 && L == 8) ? (lig >> 1) : ((lig >> (2 * (NLEAD - 1 - q))) & 3);
    piece_coeffs<T>(aq, hc[q][0], hc[q][1], hc[q][2], hc[q][3]);
    lead_off += aq * st[q];
  }
  const int hh = (D == 3 && L == 8) ? (lig & 1) : 0;   // the lane's half of dimension D-2
  if constexpr (D == 3 && L == 8) lead_off += hh * 2 * st[1];

  // level-g positions in the cell of points [from, from + m) to s_tt[p][0..m)
  auto stage_points = [&](int64_t from, int m) {
    for (int idx = threadIdx.x; idx < m; idx += kBlock) {
      const size_t i = size_t(from) + size_t(idx);
      const uint32_t cf = a.cell[i];
#pragma unroll
      for (int p = 0; p < D; ++p) {
        const uint32_t cfp = (cf >> (a.G * (D - 1 - p))) & maskN;
        s_tt[p * a.ppb + idx] = (T(double(cfp & maskSh)) + tfrac[size_t(p) * size_t(a.n) + i]) * scale;
      }
    }
  };

  const int wg = xcd_block();
  int64_t pos = 0, end = 0, seg_end = 0;
  int c_cur = 0, c_end = 0;
  // A split work list (d <= 3) gives workgroup wg exactly the points
  // [wg ppb, (wg+1) ppb): they are staged once, up front, while the chunk
  // descriptors are still loading.
  constexpr bool STAGE_ONCE = WL && D <= 3;
  int64_t wbase = 0;
  if constexpr (STAGE_ONCE) {
    wbase = int64_t(wg) * a.ppb;
    stage_points(wbase, int(min(a.n, wbase + int64_t(a.ppb)) - wbase));
  }
  if constexpr (WL) {
    c_cur = a.wl_first[wg];
    c_end = a.wl_first[wg + 1];
  } else {
    pos = int64_t(wg) * a.ppb;
    end = min(a.n, pos + int64_t(a.ppb));
  }
  int org[D];
  // With a work list the loop runs over the workgroup's chunks; the first
  // chunk of a tile segment stages the coefficient patch and clears the
  // accumulator, the last one flushes it. Without, over the tile segments of
  // the workgroup's ppb points, each one chunk.
  for (;;) {
    bool seg_first = true, seg_last = true;
    uint32_t tile;
    int item_b = 0, item_e = 0;
    if constexpr (WL) {
      if (c_cur >= c_end) break;
      const int4 cd = a.wl_chunks[c_cur];
      pos = cd.x;
      seg_end = cd.y;
      item_b = cd.z;
      item_e = a.wl_chunks[c_cur + 1].z;
      const uint32_t tw = uint32_t(cd.w);
      tile = tw & kChunkTile;
      seg_first = (tw & kChunkFirst) != 0;
      seg_last = (tw & kChunkLast) != 0;
      ++c_cur;
    } else {
      if (pos >= end) break;
      tile = a.mkey[pos] >> S;
      seg_end = min(end, int64_t(a.off[size_t(tile + 1) << S]));
      if (seg_end <= pos) break;   // offsets are monotone with off[N^D] = n; never taken
    }
    if (!seg_first) __syncthreads();   // the previous chunk's points and items are consumed

    // per-cell point ranges of this segment, cut into items of <= Q points;
    // thread j owns cell j of the tile (cells_in_tile <= kBlock)
    int nch = 0, cnt = 0, lo_rel = 0;
    if (!WL && int(threadIdx.x) < cells_in_tile) {
      const size_t gc = (size_t(tile) << (D * tbits)) + size_t(threadIdx.x);
      int64_t lo = a.off[gc << (D * sh)], hi = a.off[(gc + 1) << (D * sh)];
      lo = max(lo, pos);
      hi = min(hi, seg_end);
      cnt = hi > lo ? int(hi - lo) : 0;
      lo_rel = int(lo - pos);
      nch = (cnt + Q - 1) / Q;
    }
    // stage the chunk's points (one coalesced pass), unless staged up front
    if constexpr (!STAGE_ONCE) stage_points(pos, int(seg_end - pos));
    const int sbase = STAGE_ONCE ? int(pos - wbase) : 0;   // the chunk's first point in s_tt
    if (seg_first) {
      morton_decode<D>(tile, a.g - tbits, org);
#pragma unroll
      for (int p = 0; p < D; ++p) org[p] *= Tg;
      // the coefficient patch (once per segment); clear the accumulator
      for (int e = threadIdx.x; e < patch; e += kBlock) {
        if constexpr (MODE == kApply && STAGE_C) {
          int rem = e;
          int64_t gidx = 0;
#pragma unroll
          for (int p = 0; p < D; ++p) {
            const int l = rem / st[p];
            rem -= l * st[p];
            gidx = gidx * Jg + (org[p] + l);
          }
          lc[e] = cin[gidx];
        }
        lacc[e] = 0.0;
      }
    }
    int n_items = 0;
    if constexpr (WL) {
      // the chunk's items go to LDS with the points (at most ppb / Q +
      // cells of a tile of them), so the item loop waits on no global load
      n_items = min(item_e - item_b, maxi);
      for (int e = threadIdx.x; e < n_items; e += kBlock) s_items[e] = a.wl_items[item_b + e];
      __syncthreads();
    } else {
      int n_items_all;
      const int first = block_exclusive_scan(nch, scan_sh, &n_items_all);
      // first + k < ppb / Q + kMaxTileCells = maxi
      for (int k = 0; k < nch && first + k < maxi; ++k) {
        it_cell[first + k] = int(threadIdx.x);
        it_lo[first + k] = lo_rel + k * Q;
        it_cnt[first + k] = min(Q, cnt - k * Q);
      }
      __syncthreads();
      n_items = min(n_items_all, maxi);
    }

    // item `it` of the chunk into the lane's accumulators; returns its cell
    // (index inside the tile), with the lane's first patch entry and the
    // patch stride of dimension D-2
    auto run_item = [&](int it, T (&acc)[V], int& base, int& sa) -> int {
      int j, l0, l1;
      if constexpr (WL) {
        const uint32_t w = s_items[it];
        j = int(w & 0xFFu);
        l0 = int((w >> kItemLoShift) & 0xFFFu);
        l1 = l0 + int(w >> kItemCntShift);
      } else {
        j = it_cell[it];
        l0 = it_lo[it];
        l1 = l0 + it_cnt[it];
      }
      int cl[D];
      morton_decode<D>(uint32_t(j), tbits, cl);
      base = lead_off;
#pragma unroll
      for (int p = 0; p < D; ++p) base += cl[p] * st[p];
      sa = 0;
      if constexpr (D >= 2) sa = st[D - 2];
      T cv[V];
      if constexpr (MODE == kApply && !STAGE_C) {
        // global index of the lane's first coefficient: tile origin + local offset
        int64_t gbase = 0;
        int rem = base;
#pragma unroll
        for (int p = 0; p < D; ++p) {
          const int l = rem / st[p];
          rem -= l * st[p];
          gbase = gbase * Jg + (org[p] + l);
        }
        const int64_t gsa = (D >= 2) ? int64_t(Jg) : 0;
#pragma unroll
        for (int v = 0; v < V; ++v) cv[v] = cin[gbase + (D == 1 ? v : (v >> 2) * gsa + (v & 3))];
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int off = (D == 1) ? v : ((v >> 2) * sa + (v & 3));
        if constexpr (MODE == kApply && STAGE_C) cv[v] = lc[base + off];
        acc[v] = T(0);
      }
      // one point per step: the live registers stay low enough for six
      // (d = 3) or four (d = 4, 5) waves per SIMD, which hides the LDS and
      // DPP latencies better than two interleaved points at three waves
      for (int li = l0; li < l1; ++li) {
        PointVals<D, T> q0;
        point_basis<D, T, NLEAD>(s_tt, a.ppb, sbase + li, hc, q0);
        T s0;
        if constexpr (D == 3 && L == 8) {
          const T b2lo = hh ? q0.bm2[2] : q0.bm2[0];
          const T b2hi = hh ? q0.bm2[3] : q0.bm2[1];
          if constexpr (MODE == kApply) {
            T r0 = T(0), r1 = T(0);
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
              r0 += q0.bm1[bb] * cv[bb];
              r1 += q0.bm1[bb] * cv[4 + bb];
            }
            s0 = group_sum<T, L>(q0.w * (b2lo * r0 + b2hi * r1));
          } else if constexpr (MODE == kRhs) {
            s0 = T(a.y[pos + li]);
          } else {
            s0 = T(1);
          }
          const bool sq = MODE == kDiag;
          const T u = sq ? s0 * q0.w * q0.w : s0 * q0.w;
          const T u0 = sq ? u * b2lo * b2lo : u * b2lo;
          const T u1 = sq ? u * b2hi * b2hi : u * b2hi;
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) {
            acc[bb] += sq ? u0 * q0.bm1[bb] * q0.bm1[bb] : u0 * q0.bm1[bb];
            acc[4 + bb] += sq ? u1 * q0.bm1[bb] * q0.bm1[bb] : u1 * q0.bm1[bb];
          }
        } else {
        if constexpr (MODE == kApply) s0 = group_sum<T, L>(q0.w * point_gather<D, T>(q0, cv));
        else if constexpr (MODE == kRhs) s0 = T(a.y[pos + li]);
        else s0 = T(1);
        point_scatter<D, T, MODE == kDiag>(q0, s0, acc);
        }
      }
      return j;
    };

    if constexpr (!DET) {
      for (int it = grp; it < n_items; it += GP::NG) {
        T acc[V];
        int base, sa;
        run_item(it, acc, base, sa);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int off = (D == 1) ? v : ((v >> 2) * sa + (v & 3));
          atomicAdd(&lacc[base + off], double(acc[v]));
        }
      }
    } else {
      // rounds of one item per lane group; after each, every patch entry
      // adds the contributions of the round's items that cover it, in lane
      // group order
      const int rounds = (n_items + GP::NG - 1) / GP::NG;
      for (int rd = 0; rd < rounds; ++rd) {
        const int it = rd * GP::NG + grp;
        T acc[V];
        int jc = -1;
        if (it < n_items) {
          int base, sa;
          jc = run_item(it, acc, base, sa);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) acc[v] = T(0);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) s_slot[size_t(threadIdx.x) * V + v] = double(acc[v]);
        if (lig == 0) {
          // the item's cell as packed tile coordinates, 6 bits per dimension
          int pc = -1;
          if (jc >= 0) {
            int cl[D];
            morton_decode<D>(uint32_t(jc), tbits, cl);
            pc = 0;
#pragma unroll
            for (int p = 0; p < D; ++p) pc |= cl[p] << (6 * p);
          }
          s_jcell[grp] = pc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < patch; e += kBlock) {
          int el[D];
          {
            int rem = e;
#pragma unroll
            for (int p = 0; p < D; ++p) {
              el[p] = rem / st[p];
              rem -= el[p] * st[p];
            }
          }
          double sum = 0.0;
          for (int g2 = 0; g2 < GP::NG; ++g2) {
            const int pc = s_jcell[g2];
            if (pc < 0) continue;
            bool in = true;
            int dl[D];
#pragma unroll
            for (int p = 0; p < D; ++p) {
              dl[p] = el[p] - ((pc >> (6 * p)) & 63);
              in = in && unsigned(dl[p]) <= unsigned(kDeg);
            }
            if (!in) continue;
            int lane = 0, v;
            if constexpr (D == 3 && L == 8) {
              // eight lanes: the leading digit and the half of dimension 1
              lane = dl[0] * 2 + (dl[1] >> 1);
              v = (dl[1] & 1) * 4 + dl[2];
            } else if constexpr (D == 1) {
              v = dl[0];
            } else {
#pragma unroll
              for (int q = 0; q < NLEAD; ++q) lane = lane * 4 + dl[q];
              v = dl[D - 2] * 4 + dl[D - 1];
            }
            sum += s_slot[(size_t(g2) * L + lane) * V + v];
          }
          lacc[e] += sum;
        }
        __syncthreads();
      }
    }
    if (!seg_last) continue;
    __syncthreads();

    if constexpr (DET) {
      // the segment is this one chunk (c_cur - 1): its patch to det_part
      double* dst = a.det_part + size_t(c_cur - 1) * size_t(patch);
      for (int e = threadIdx.x; e < patch; e += kBlock) dst[e] = lacc[e];
    } else for (int e = threadIdx.x; e < patch; e += kBlock) {
      const T v = T(lacc[e]);
      if (v != T(0)) {
        int rem = e;
        int64_t gidx = 0;
#pragma unroll
        for (int p = 0; p < D; ++p) {
          const int l = rem / st[p];
          rem -= l * st[p];
          gidx = gidx * Jg + (org[p] + l);
        }
        atomicAdd(&out[gidx], v);
      }
    }
    __syncthreads();
    if constexpr (!WL) pos = seg_end;
  }
}


// The second half of the reproducible point pass: out[k] += the sum of the
// stored patches that cover coefficient k - per dimension the one or two
// tiles whose (2^tb + 3)-wide patch contains k, their combinations in a fixed
// order, each tile's chunks in increasing order. One writer per entry.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_det_reduce(const double* part, const int32_t* tile_first, T* out,
                                                       int g, int tb, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  const int J = (1 << g) + kDeg, Tg = 1 << tb, P = Tg + kDeg, ntp = 1 << (g - tb);
  int patch = 1;
#pragma unroll
  for (int p = 0; p < D; ++p) patch *= P;
  int j[D];
  {
    int64_t rem = k;
#pragma unroll
    for (int p = D - 1; p >= 0; --p) {
      j[p] = int(rem % J);
      rem /= J;
    }
  }
  int tc[D][2], nc[D], idx[D];
#pragma unroll
  for (int p = 0; p < D; ++p) {
    nc[p] = 0;
    idx[p] = 0;
    const int tA = min(j[p] >> tb, ntp - 1);
    for (int t = tA; t >= 0 && t >= tA - 1; --t) {
      const int o = j[p] - t * Tg;
      if (o >= 0 && o <= Tg + kDeg - 1) tc[p][nc[p]++] = t;
    }
  }
  double sum = 0.0;
  for (;;) {
    uint32_t key = 0;
    int e = 0;
#pragma unroll
    for (int p = 0; p < D; ++p) {
      const int t = tc[p][idx[p]];
      e = e * P + (j[p] - t * Tg);
      for (int b = 0; b < g - tb; ++b) key |= uint32_t((t >> b) & 1) << (b * D + (D - 1 - p));
    }
    for (int c = tile_first[key]; c < tile_first[key + 1]; ++c) sum += part[size_t(c) * size_t(patch) + size_t(e)];
    int p = D - 1;
    while (p >= 0 && ++idx[p] == nc[p]) {
      idx[p] = 0;
      --p;
    }
    if (p < 0) break;
  }
  out[k] = T(double(out[k]) + sum);
}

// ---------------------------------------------------------------------------
// lambda * Lambda_g c by the three-accumulator sum factorisation of
// Lambda = sum_p (M x..x G2_p x..x M) + 2 sum_{p<q} (M x..G1_p..G1_q..x M):
// after processing dimensions 0..p the tensors hold
//   T0 = (M x..x M) c, T1 = sum of one G1 factor, T2 = Lambda restricted to the
// processed dimensions; one pass applies along dimension p
//   T2' = M T2 + G2 T0 + 2 G1 T1,  T1' = M T1 + G1 T0,  T0' = M T0.
// `band` holds three J x 7 banded factors (M, G1, G2), row j column j+o-3.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lambda_pass(LambdaArgs<T> a) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= a.K) return;
  const int64_t S = a.stride;
  const int jp = int((k / S) % a.J);
  const T* m = a.band + size_t(jp) * 7;
  const T* g1 = a.band + size_t(a.J) * 7 + size_t(jp) * 7;
  const T* g2 = a.band + size_t(2 * a.J) * 7 + size_t(jp) * 7;
  T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
  for (int o = -3; o <= 3; ++o) {
    const int jj = jp + o;
    if (jj < 0 || jj >= a.J) continue;
    const int64_t idx = k + int64_t(o) * S;
    const T v0 = a.in0[idx];
    const T mm = m[o + 3], gg1 = g1[o + 3], gg2 = g2[o + 3];
    if (a.first) {
      s0 += mm * v0;
      s1 += gg1 * v0;
      s2 += gg2 * v0;
    } else {
      const T v1 = a.in1[idx], v2 = a.in2[idx];
      s0 += mm * v0;
      s1 += mm * v1 + gg1 * v0;
      s2 += mm * v2 + gg2 * v0 + T(2) * gg1 * v1;
    }
  }
  if (a.last) {
    a.out[k] = a.lam * s2;
  } else {
    a.out0[k] = s0;
    a.out1[k] = s1;
    a.out2[k] = s2;
  }
}

// lambda * Lambda c in one kernel for d = 2 and 3, running the
// three-accumulator recursion of k_lambda_pass over the dimensions on chip
// (out-of-grid entries of c are zero, which drops the same taps the pass form
// skips). band: d blocks of [3][J][7] (M, G1, G2 per dimension).
//
// Last three dimensions (all three at d = 3; at d >= 4 after k_lambda_pass
// has run the leading ones, which leaves three tensors T0, T1, T2): a
// workgroup owns a kLamT x kLamT column tile in the last two dimensions
// (halo included, so kLamB = kLamT - 6 outputs per edge), a run of C0 output
// planes along the third-to-last dimension and one index of the leading
// dimensions (`outer`, each a J^3 block). Each thread loads its column of
// the input(s) over the run and its halo into registers once; then, kLamP
// planes at a time, the first contraction happens in registers and the
// other two go through LDS (two barriers per kLamP planes; the planes of a
// step are independent, which hides LDS latency). Every input entry is read
// (kLamT / kLamB)^2 (C0 + 6) / C0 times, from L2 mostly.
constexpr int kLamT = 16;
constexpr int kLamB = kLamT - 6;
constexpr int kLamC0 = 8;    // planes per run, one input tensor (d = 3)
constexpr int kLamC0x3 = 4;  // planes per run, three input tensors (d >= 4)
constexpr int kLamP = 2;
constexpr int kLamS = kLamT + 1;   // LDS row stride after the second dimension (odd: rows fall on different banks)
static_assert(kLamT * kLamT == kBlock, "one thread per column of the tile");
static_assert(kLamC0 % kLamP == 0 && kLamC0x3 % kLamP == 0, "whole steps per run");

template <typename T>
__device__ __forceinline__ void band_row(const T* band, int J, int j, T (&m)[7], T (&g1)[7], T (&g2)[7]) {
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    m[o] = band[size_t(j) * 7 + o];
    g1[o] = band[size_t(J) * 7 + size_t(j) * 7 + o];
    g2[o] = band[size_t(2 * J) * 7 + size_t(j) * 7 + o];
  }
}

// c0, c1, c2: the input tensors (c1, c2 read only when THREE); band: the
// factors of the last three dimensions, [3][3][J][7].
template <typename T, bool THREE, int C0>
__global__ __launch_bounds__(kBlock) void k_lambda_fused3(const T* __restrict__ c0, const T* __restrict__ c1,
                                                          const T* __restrict__ c2, T* __restrict__ out,
                                                          const T* __restrict__ band, int J, int B, int nt, int nt0,
                                                          T lam) {
  __shared__ T s1[kLamP][3][kLamT * kLamT];   // T0, T1, T2 after the first dimension, per column
  __shared__ T s2[kLamP][3][kLamB * kLamS];   // after the second
  __shared__ T sb[3][C0][7];                  // first-dimension band rows (M, G1, G2) of the run
  const int wg = xcd_block();   // an XCD takes whole runs of planes: the halos stay in its L2
  const int t2 = wg % nt;
  const int t1 = (wg / nt) % nt;
  const int z0 = ((wg / (nt * nt)) % nt0) * C0;
  const int64_t JJ = int64_t(J) * J;
  const int64_t base = int64_t(wg / (nt * nt * nt0)) * JJ * J;   // the outer block
  const int tid = threadIdx.x;
  T v0[C0 + 6], v1[THREE ? C0 + 6 : 1], v2[THREE ? C0 + 6 : 1];
  {
    const int g1 = t1 * B - 3 + tid / kLamT, g2 = t2 * B - 3 + tid % kLamT;
    const bool col = g1 >= 0 && g1 < J && g2 >= 0 && g2 < J;
#pragma unroll
    for (int i = 0; i < C0 + 6; ++i) {
      const int g0 = z0 - 3 + i;
      const bool ok = col && g0 >= 0 && g0 < J;
      const int64_t idx = base + int64_t(g0) * JJ + int64_t(g1) * J + g2;
      v0[i] = ok ? c0[idx] : T(0);
      if constexpr (THREE) {
        v1[i] = ok ? c1[idx] : T(0);
        v2[i] = ok ? c2[idx] : T(0);
      }
    }
  }
  // second dimension: thread -> (row b1a of the output tile, column h2a);
  // third: thread -> output (b1b, b2b)
  const int b1a = tid / kLamT, h2a = tid % kLamT;
  const int b1b = tid / B, b2b = tid % B;
  const bool do1 = b1a < B && t1 * B + b1a < J;
  const bool do2 = b1b < B && t1 * B + b1b < J && t2 * B + b2b < J;
  T m1[7], p1[7], q1[7], m2[7], p2[7], q2[7];
  band_row(band + size_t(3) * J * 7, J, do1 ? t1 * B + b1a : 0, m1, p1, q1);
  band_row(band + size_t(6) * J * 7, J, do2 ? t2 * B + b2b : 0, m2, p2, q2);
  const int nsteps = min(C0, J - z0);
  for (int e = tid; e < 3 * C0 * 7; e += kBlock) {
    const int kind = e / (C0 * 7), i = (e / 7) % C0, o = e % 7;
    sb[kind][i][o] = i < nsteps ? band[(size_t(kind) * J + z0 + i) * 7 + o] : T(0);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < C0; i += kLamP) {
    if (i >= nsteps) break;
#pragma unroll
    for (int p = 0; p < kLamP; ++p) {
      T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
      for (int o = 0; o < 7; ++o) {
        const T m = sb[0][i + p][o], g1 = sb[1][i + p][o], g2 = sb[2][i + p][o];
        if constexpr (THREE) {
          a0 += m * v0[i + p + o];
          a1 += m * v1[i + p + o] + g1 * v0[i + p + o];
          a2 += m * v2[i + p + o] + g2 * v0[i + p + o] + T(2) * g1 * v1[i + p + o];
        } else {
          a0 += m * v0[i + p + o];
          a1 += g1 * v0[i + p + o];
          a2 += g2 * v0[i + p + o];
        }
      }
      s1[p][0][tid] = a0;
      s1[p][1][tid] = a1;
      s1[p][2][tid] = a2;
    }
    __syncthreads();   // s1 complete; the previous step's readers of s2 are done
    if (do1) {
#pragma unroll
      for (int p = 0; p < kLamP; ++p) {
        T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll
        for (int o = 0; o < 7; ++o) {
          const int q = (b1a + o) * kLamT + h2a;
          const T w0 = s1[p][0][q], w1 = s1[p][1][q], w2 = s1[p][2][q];
          a0 += m1[o] * w0;
          a1 += m1[o] * w1 + p1[o] * w0;
          a2 += m1[o] * w2 + q1[o] * w0;
          a3 += p1[o] * w1;
        }
        s2[p][0][b1a * kLamS + h2a] = a0;
        s2[p][1][b1a * kLamS + h2a] = a1;
        s2[p][2][b1a * kLamS + h2a] = a2 + T(2) * a3;
      }
    }
    __syncthreads();   // s2 complete; every reader of s1 is done
    if (do2) {
#pragma unroll
      for (int p = 0; p < kLamP; ++p) {
        if (i + p >= nsteps) break;
        T a = T(0), b = T(0);
#pragma unroll
        for (int o = 0; o < 7; ++o) {
          const int q = b1b * kLamS + b2b + o;
          a += m2[o] * s2[p][2][q] + q2[o] * s2[p][0][q];
          b += p2[o] * s2[p][1][q];
        }
        out[base + int64_t(z0 + i + p) * JJ + int64_t(t1 * B + b1b) * J + (t2 * B + b2b)] = lam * (a + T(2) * b);
      }
    }
  }
}

// d = 2: a workgroup stages a halo-extended kLam2H0 x kLam2H1 tile of c in
// LDS and runs both passes there.
constexpr int kLam2B0 = 8, kLam2B1 = 32;
constexpr int kLam2H0 = kLam2B0 + 6, kLam2H1 = kLam2B1 + 6;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_lambda_fused2(const T* c, T* out, const T* band, int J, int B0, int B1,
                                                          int nt1, T lam) {
  __shared__ T sin_[kLam2H0 * kLam2H1];
  __shared__ T s1[3 * kLam2B0 * kLam2H1];
  const int t1 = blockIdx.x % nt1;
  const int t0 = blockIdx.x / nt1;
  const int H0 = B0 + 6, H1 = B1 + 6;
  const int b0base = t0 * B0 - 3, b1base = t1 * B1 - 3;
  for (int e = threadIdx.x; e < H0 * H1; e += kBlock) {
    const int h1 = e % H1, h0 = e / H1;
    const int g0 = b0base + h0, g1 = b1base + h1;
    const bool ok = g0 >= 0 && g0 < J && g1 >= 0 && g1 < J;
    sin_[e] = ok ? c[int64_t(g0) * J + g1] : T(0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < B0 * H1; e += kBlock) {
    const int h1 = e % H1, b0 = e / H1;
    const int j0 = t0 * B0 + b0;
    if (j0 >= J) continue;
    T m[7], g1c[7], g2c[7];
    band_row(band, J, j0, m, g1c, g2c);
    T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
    for (int o = 0; o < 7; ++o) {
      const T v = sin_[(b0 + o) * H1 + h1];
      a0 += m[o] * v;
      a1 += g1c[o] * v;
      a2 += g2c[o] * v;
    }
    s1[e] = a0;
    s1[B0 * H1 + e] = a1;
    s1[2 * B0 * H1 + e] = a2;
  }
  __syncthreads();
  const T* band1 = band + size_t(3) * J * 7;
  for (int e = threadIdx.x; e < B0 * B1; e += kBlock) {
    const int b1 = e % B1, b0 = e / B1;
    const int j0 = t0 * B0 + b0, j1 = t1 * B1 + b1;
    if (j0 >= J || j1 >= J) continue;
    T m[7], g1c[7], g2c[7];
    band_row(band1, J, j1, m, g1c, g2c);
    T a = T(0);
#pragma unroll
    for (int o = 0; o < 7; ++o) {
      const int q = b0 * H1 + b1 + o;
      a += m[o] * s1[2 * B0 * H1 + q] + g2c[o] * s1[q] + T(2) * g1c[o] * s1[B0 * H1 + q];
    }
    out[int64_t(j0) * J + j1] = lam * a;
  }
}

// lambda * diag(Lambda_g) from the diagonals of the 1D factors; `band` holds
// [D][3][J][7] (each dimension has its own mesh width).
template <int D>
__global__ __launch_bounds__(kBlock) void k_lambda_diag(const double* band, int J, int64_t K,
                                                        double lam, double* out) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  double md[D], g1d[D], g2d[D];
  int64_t rem = k;
#pragma unroll
  for (int p = D - 1; p >= 0; --p) {
    const int j = int(rem % J);
    rem /= J;
    const double* bp = band + size_t(p) * 3 * J * 7;   // dimension p's factors
    md[p] = bp[size_t(j) * 7 + 3];
    g1d[p] = bp[size_t(J) * 7 + size_t(j) * 7 + 3];
    g2d[p] = bp[size_t(2 * J) * 7 + size_t(j) * 7 + 3];
  }
  double total = 0.0;
#pragma unroll
  for (int p = 0; p < D; ++p) {
    double t = g2d[p];
#pragma unroll
    for (int q = 0; q < D; ++q)
      if (q != p) t *= md[q];
    total += t;
  }
#pragma unroll
  for (int p = 0; p < D; ++p)
#pragma unroll
    for (int q = p + 1; q < D; ++q) {
      double t = 2.0 * g1d[p] * g1d[q];
#pragma unroll
      for (int r = 0; r < D; ++r)
        if (r != p && r != q) t *= md[r];
      total += t;
    }
  out[k] = lam * total;
}

// ---------------------------------------------------------------------------
// Grid transfer, one dimension per pass (Alg. 2 with the 1D subdivision
// matrix of eq. 2.5, 0-based I[i, j] = binom(4, i - 2j + 3) / 8):
// prolongation expands dimension p from Jc to Jf = 2 Jc - 3, restriction
// contracts it back with the transposed weights.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_pass(TransferArgs<T> a) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= a.Kout) return;
  const int64_t inner = a.inner;
  const int64_t ii = k % inner;
  const int64_t rest = k / inner;
  const int i = int(rest % a.Jf);
  const int64_t outer = rest / a.Jf;
  const int64_t ibase = outer * a.Jc * inner + ii;
  T v;
  const int mm = i >> 1;
  if (i & 1) {
    v = T(0.125) * a.in[ibase + int64_t(mm) * inner];
    if (mm + 1 < a.Jc) v += T(0.75) * a.in[ibase + int64_t(mm + 1) * inner];
    if (mm + 2 < a.Jc) v += T(0.125) * a.in[ibase + int64_t(mm + 2) * inner];
  } else {
    v = T(0.5) * a.in[ibase + int64_t(mm) * inner];
    if (mm + 1 < a.Jc) v += T(0.5) * a.in[ibase + int64_t(mm + 1) * inner];
  }
  if (a.subtract) a.out[k] -= v;
  else a.out[k] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_pass(TransferArgs<T> a) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= a.Kout) return;
  const int64_t inner = a.inner;
  const int64_t ii = k % inner;
  const int64_t rest = k / inner;
  const int j = int(rest % a.Jc);
  const int64_t outer = rest / a.Jc;
  const int64_t ibase = outer * a.Jf * inner + ii;
  const T w[5] = {T(0.125), T(0.5), T(0.75), T(0.5), T(0.125)};
  T v = T(0);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const int i = 2 * j - 3 + m;
    if (i >= 0 && i < a.Jf) {
      const int64_t idx = ibase + int64_t(i) * inner;
      v += w[m] * (a.sub ? a.in[idx] - a.sub[idx] : a.in[idx]);
    }
  }
  a.out[k] = v;
  if (a.a) a.a[k] = a.w[k] * v;
}

// ---------------------------------------------------------------------------
// Jacobi smoother and residual epilogues (Alg. 6, Alg. 7).
// All d dimensions of a transfer in one kernel, for small levels where the
// pass-per-dimension form is launch-bound. Per dimension each output takes
// up to 5 (restriction) or 3 (prolongation) inputs; idx holds their flat
// offsets (stride included) and wt their weights (0 for indices that fall
// off the grid, whose offset is then 0).
template <int D, int P, int M, typename T>
struct TensorGather {
  static __device__ __forceinline__ T sum(const T* in, const T* sub, const int64_t (&idx)[D][M],
                                          const T (&wt)[D][M], int64_t off) {
    T v = T(0);
#pragma unroll
    for (int m = 0; m < M; ++m)
      if (wt[P][m] != T(0)) v += wt[P][m] * TensorGather<D, P + 1, M, T>::sum(in, sub, idx, wt, off + idx[P][m]);
    return v;
  }
};
template <int D, int M, typename T>
struct TensorGather<D, D, M, T> {
  static __device__ __forceinline__ T sum(const T* in, const T* sub, const int64_t (&)[D][M], const T (&)[D][M],
                                          int64_t off) {
    return sub ? in[off] - sub[off] : in[off];
  }
};

// out (coarse, Jc^D) = (I_{g-1}^g)' (in - sub) (sub may be null). Each coarse
// entry gathers 5^D fine entries; 32 lanes share them and sum by shuffles,
// 8 coarse entries per workgroup.
constexpr int kRestrictLanes = 32;

template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_fused(const T* in, const T* sub, T* out, int Jc, int Jf,
                                                           int64_t Kc, const T* wj, T* aj) {
  constexpr int NT = (D == 1) ? 5 : (D == 2 ? 25 : (D == 3 ? 125 : 625));
  const int lane = threadIdx.x % kRestrictLanes;
  const int64_t k = int64_t(blockIdx.x) * (kBlock / kRestrictLanes) + threadIdx.x / kRestrictLanes;
  int j[D];
  {
    int64_t rem = k < Kc ? k : 0;
#pragma unroll
    for (int p = D - 1; p >= 0; --p) {
      j[p] = int(rem % Jc);
      rem /= Jc;
    }
  }
  T v = T(0);
  if (k < Kc) {
    for (int t = lane; t < NT; t += kRestrictLanes) {
      int rem = t;
      int64_t off = 0;
      T w = T(1);
      bool ok = true;
#pragma unroll
      for (int p = D - 1; p >= 0; --p) {
        const int m = rem % 5;
        rem /= 5;
        const int i = 2 * j[p] - 3 + m;
        ok = ok && i >= 0 && i < Jf;
        w *= (m == 0 || m == 4) ? T(0.125) : (m == 2 ? T(0.75) : T(0.5));
        int64_t stride = 1;
#pragma unroll
        for (int q = p + 1; q < D; ++q) stride *= Jf;
        off += int64_t(i) * stride;
      }
      if (ok) v += w * (sub ? in[off] - sub[off] : in[off]);
    }
  }
#pragma unroll
  for (int m = kRestrictLanes / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  if (lane == 0 && k < Kc) {
    out[k] = v;
    if (aj) aj[k] = wj[k] * v;   // the coarse level's first Jacobi sweep from zero
  }
}

// out (fine, Jf^D) = I_{g-1}^g e, or out -= I_{g-1}^g e when subtract is set.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_fused(const T* e, T* out, int Jc, int Jf, int64_t Kf,
                                                          int subtract) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= Kf) return;
  int64_t idx[D][3];
  T wt[D][3];
  int64_t rem = k, stride = 1;
#pragma unroll
  for (int p = D - 1; p >= 0; --p) {
    const int i = int(rem % Jf);
    rem /= Jf;
    const int mm = i >> 1;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int j = mm + m;
      T w;
      if (i & 1) w = (m == 1) ? T(0.75) : T(0.125);
      else w = (m == 2) ? T(0) : T(0.5);
      const bool ok = j < Jc && w != T(0);
      wt[p][m] = ok ? w : T(0);
      idx[p][m] = ok ? int64_t(j) * stride : 0;
    }
    stride *= Jc;
  }
  const T v = TensorGather<D, 0, 3, T>::sum(e, static_cast<const T*>(nullptr), idx, wt, 0);
  if (subtract) out[k] -= v;
  else out[k] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_first(T* alpha, const T* wdinv, const T* b, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) alpha[k] = wdinv[k] * b[k];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi(T* alpha, const T* wdinv, const T* b, const T* Ax, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) alpha[k] += wdinv[k] * (b[k] - Ax[k]);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual(T* r, const T* Ax, const T* b, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) r[k] = Ax[k] - b[k];
}

// ---------------------------------------------------------------------------
// Vector kernels. Reductions accumulate in FP64 whatever the input type and
// are two-stage (per-block partials, then one block) so results do not depend
// on scheduling.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

template <typename TX, typename TY>
__global__ __launch_bounds__(kBlock) void k_dot_partial(const TX* x, const TY* y, int64_t K, double* partial) {
  __shared__ double sh[kBlock / 64];
  double v = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < K; k += int64_t(gridDim.x) * kBlock)
    v += double(x[k]) * double(y[k]);
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* partial, int nb, double* slot) {
  __shared__ double sh[kBlock / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) v += partial[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) *slot = v;
}

// The second stage of a reduction whose first stage wrote NV rows of nb
// per-block partials (row j at partial + j * kMaxPartials): *slot[j] is the
// sum of row j in index order.
__global__ __launch_bounds__(kBlock) void k_sum_rows(const double* partial, int nb, int nv, double* slot0,
                                                     double* slot1) {
  __shared__ double sh[kBlock / 64];
  for (int j = 0; j < nv; ++j) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) v += partial[j * kMaxPartials + i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) *(j == 0 ? slot0 : slot1) = v;
  }
}

// The second stage of a reduction inside the kernel that consumes it: every
// block sums the nb first-stage partials itself, in the order k_sum_partials
// takes (so every block, and the slot, get the same bits), and block 0
// stores the total in *out for the host and later kernels.
__device__ __forceinline__ double resum(const double* partial, int nb, double* out, double* sh, double* bc) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) v += partial[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) {
    *bc = v;
    if (blockIdx.x == 0) *out = v;
  }
  __syncthreads();
  return *bc;
}

// alpha += w p; r -= w v with w = (*num) / (*den) read on the device. A step
// with den <= 0 (a breakdown, which the host reports) leaves both unchanged.
template <typename TA, typename T>
__global__ __launch_bounds__(kBlock) void k_cg_step(TA* alpha, T* r, const T* p, const T* v, int64_t K,
                                                    const double* num, const double* den) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  const double dn = *den;
  if (!(dn > 0.0) || !isfinite(dn)) return;
  const double w = *num / dn;
  alpha[k] = TA(double(alpha[k]) + w * double(p[k]));
  r[k] = T(double(r[k]) - w * double(v[k]));
}

// The FP64 CG step fused with the first stage of the norms the iteration
// needs next: alpha += w p; r -= w v (w = (*num) / (*den)), and per block the
// partial sums of r'r (row 0) and, when z is given, of r'z (row 1: the new
// residual against the previous preconditioned one, for the flexible
// direction update), in the same per-block split as k_dot_partial; with zf
// given it also writes zf = wz .* r, the first Jacobi sweep of the V-cycle
// that preconditions r next (zf may be z: each entry is read before it is
// written). A step with den <= 0 leaves alpha and r unchanged (the host
// reports the breakdown). With den_part given, den is the sum of its nb
// partials (p'v, the first stage of its reduction), stored to *den.
__global__ __launch_bounds__(kBlock) void k_cg_step_norms(double* alpha, double* r, const double* p, const double* v,
                                                          const double* z, int64_t K, const double* num,
                                                          double* den, double* partial, const double* wz,
                                                          double* zf, const double* den_part, int den_nb) {
  __shared__ double sh[kBlock / 64];
  __shared__ double bc;
  const double dn = den_part ? resum(den_part, den_nb, den, sh, &bc) : *den;
  const bool ok = dn > 0.0 && isfinite(dn);
  const double w = ok ? *num / dn : 0.0;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < K; k += int64_t(gridDim.x) * kBlock) {
    double rk = r[k];
    if (ok) {
      alpha[k] += w * p[k];
      rk -= w * v[k];
      r[k] = rk;
    }
    a0 += rk * rk;
    if (z) a1 += rk * z[k];
    if (zf) zf[k] = wz[k] * rk;
  }
  a0 = block_sum(a0, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = a0;
  if (z) {
    a1 = block_sum(a1, sh);
    if (threadIdx.x == 0) partial[kMaxPartials + blockIdx.x] = a1;
  }
}

// p = z + beta p with beta = (*num) / (*den).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_p_update(T* p, const T* z, int64_t K, const double* num,
                                                     const double* den) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  const double beta = *num / *den;
  p[k] = T(double(z[k]) + beta * double(p[k]));
}

// p = z + beta p, FP64, with beta = (num - (*sub)) / (*den) (sub null: 0) and
// num the sum of the nb partials num_part (r'z), stored to *num.
__global__ __launch_bounds__(kBlock) void k_p_update_sum(double* p, const double* z, int64_t K, double* num,
                                                         const double* num_part, int nb, const double* sub,
                                                         const double* den) {
  __shared__ double sh[kBlock / 64];
  __shared__ double bc;
  const double nm = resum(num_part, nb, num, sh, &bc);
  const double beta = (sub ? nm - *sub : nm) / *den;
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) p[k] = z[k] + beta * p[k];
}

// y = (*smul)^(1/2) * x with conversion.
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scale_mul(const TI* x, TO* y, int64_t K, const double* smul) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  y[k] = TO(sqrt(*smul) * double(x[k]));
}

// y = s * x with conversion; s = scale * (*sden)^(-1/2) when sden is given.
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scale_copy(const TI* x, TO* y, int64_t K, double scale,
                                                       const double* sden) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  double s = scale;
  if (sden) s = s / sqrt(*sden);
  y[k] = TO(s * double(x[k]));
}

// y += s * x (x converted to y's type), s as in k_scale_copy but multiplied.
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_axpy_conv(const TI* x, TO* y, int64_t K, double scale,
                                                      const double* smul) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  double s = scale;
  if (smul) s = s * sqrt(*smul);
  y[k] = TO(double(y[k]) + s * double(x[k]));
}

// Lanczos pieces with device-resident scalars: y = d .* x;
// w = d .* (A y) - beta v_prev with beta = sqrt(*b2prev) (0 without b2prev);
// y += (scale * (*s)) x.
__global__ __launch_bounds__(kBlock) void k_mul(const double* d, const double* x, double* y, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) y[k] = d[k] * x[k];
}
__global__ __launch_bounds__(kBlock) void k_lanczos_w(const double* d, const double* Ax, const double* vprev,
                                                      const double* b2prev, double* w, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= K) return;
  const double beta = b2prev ? sqrt(*b2prev) : 0.0;
  w[k] = d[k] * Ax[k] - beta * vprev[k];
}
__global__ __launch_bounds__(kBlock) void k_axpy(double scale, const double* s, const double* x, double* y, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) y[k] += (scale * *s) * x[k];
}
__global__ __launch_bounds__(kBlock) void k_start_vector(double* u, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) {
    const uint64_t h = (uint64_t(k) * 2654435761ull) & 0xffffffffull;
    u[k] = double(h) / 4294967296.0 - 0.5;
  }
}
__global__ __launch_bounds__(kBlock) void k_rsqrt_vec(const double* D, double* out, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) out[k] = 1.0 / sqrt(D[k]);
}
__global__ __launch_bounds__(kBlock) void k_wdinv(const double* D, double omega, double* w64, float* w32,
                                                  int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) {
    const double v = omega / D[k];
    w64[k] = v;
    w32[k] = float(v);
  }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* x, T v, int64_t K) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K) x[k] = v;
}
// Sets nonfinite/flag bits: 1 if any value is not finite.
__global__ __launch_bounds__(kBlock) void k_check_finite(const double* x, int64_t K, int* flag) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < K && !isfinite(x[k])) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Setup: bin every point into its finest knot cell (reading: c = min(floor(
// (x - lo) / h), N - 1)), record the Morton key of the cell for the sort and
// flag non-finite or out-of-box coordinates.
template <int D>
__global__ __launch_bounds__(kBlock) void k_bin(const double* x, int64_t n, BoxArgs box, uint32_t* key,
                                                uint32_t* idx, int* flag) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  uint32_t k = 0;
  int bad = 0;
  const uint32_t N = 1u << box.G;
  uint32_t c[D];
#pragma unroll
  for (int p = 0; p < D; ++p) {
    const double xv = x[size_t(i) * D + p];
    if (!isfinite(xv)) { bad |= 2; c[p] = 0; continue; }
    if (xv < box.lo[p] || xv > box.hi[p]) { bad |= 4; c[p] = 0; continue; }
    const double u = (xv - box.lo[p]) * box.inv_h[p];
    int64_t ci = int64_t(floor(u));
    ci = ci < 0 ? 0 : (ci > int64_t(N) - 1 ? int64_t(N) - 1 : ci);
    c[p] = uint32_t(ci);
  }
  for (int b = 0; b < box.G; ++b)
#pragma unroll
    for (int p = 0; p < D; ++p) k |= ((c[p] >> b) & 1u) << (b * D + (D - 1 - p));
  key[i] = k;
  idx[i] = uint32_t(i);
  if (bad) atomicOr(flag, bad);
}

// Gather the sorted points into structure-of-arrays storage.
template <int D>
__global__ __launch_bounds__(kBlock) void k_place(const double* x, const double* y, const uint32_t* idx,
                                                  int64_t n, BoxArgs box, double* t64, float* t32,
                                                  uint32_t* cell, double* ys) {
  const int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= n) return;
  const int64_t i = idx[s];
  const int64_t N = int64_t(1) << box.G;
  uint32_t cf = 0;
#pragma unroll
  for (int p = 0; p < D; ++p) {
    const double u = (x[size_t(i) * D + p] - box.lo[p]) * box.inv_h[p];
    int64_t ci = int64_t(floor(u));
    ci = ci < 0 ? 0 : (ci > N - 1 ? N - 1 : ci);
    double t = u - double(ci);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    t64[size_t(p) * n + s] = t;
    t32[size_t(p) * n + s] = float(t);
    cf = cf * uint32_t(N) + uint32_t(ci);
  }
  cell[s] = cf;
  ys[s] = y[i];
}

// off[c] = first sorted position whose key is >= c, c = 0..ncells.
__global__ __launch_bounds__(kBlock) void k_offsets(const uint32_t* key, int64_t n, int64_t ncells,
                                                    int32_t* off) {
  const int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (c > ncells) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(key[mid]) < c) lo = mid + 1; else hi = mid;
  }
  off[c] = int32_t(lo);
}

// ---------------------------------------------------------------------------
// s(x) at query points (eq. 2.2): cell of each query on the finest grid,
// 1D cubic values, tensor gather from global memory.
template <int D>
__global__ __launch_bounds__(kBlock) void k_eval(const double* alpha, const double* xq, int64_t m,
                                                 BoxArgs box, double* yq) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= m) return;
  const int N = 1 << box.G;
  const int J = N + kDeg;
  int st[D];
  st[D - 1] = 1;
#pragma unroll
  for (int p = D - 2; p >= 0; --p) st[p] = st[p + 1] * J;
  double B[D][4];
  int base = 0;
#pragma unroll
  for (int p = 0; p < D; ++p) {
    const double u = (xq[size_t(i) * D + p] - box.lo[p]) * box.inv_h[p];
    double fl = floor(u);
    fl = fl < 0.0 ? 0.0 : (fl > double(N - 1) ? double(N - 1) : fl);
    cubic_basis(u - fl, B[p]);
    base += int(fl) * st[p];
  }
  yq[i] = patch_gather<D, double>(alpha, base, B, st);
}

// ---------------------------------------------------------------------------
// Coarse matrix A_1 (Sec. 3.2.4): the dense K_1 x K_1 matrix expanded from
// the level-1 stencil (A1 zeroed first), then inverted by Gauss-Jordan. The
// stencil holds the upper half of the offsets (see k_stencil_finalize); each
// entry fills A[k][l] and its mirror A[l][k].
template <int D>
__global__ __launch_bounds__(kBlock) void k_dense_from_stencil(const double* S, int J, int64_t K, double* A) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  int NO = 1;
#pragma unroll
  for (int p = 0; p < D; ++p) NO *= 7;
  const int NH = (NO + 1) / 2;
  if (t >= int64_t(NH) * K) return;
  const int oidx = NO / 2 + int(t / K);
  const int64_t k = t % K;
  int64_t rk = k, l = 0, stride = 1;
  int ro = oidx;
  bool inside = true;
#pragma unroll
  for (int p = D - 1; p >= 0; --p) {
    const int kp = int(rk % J), op = ro % 7 - 3;
    rk /= J;
    ro /= 7;
    inside = inside && kp + op >= 0 && kp + op < J;
    l += (kp + op) * stride;
    stride *= J;
  }
  if (inside) {
    A[k * K + l] = S[t];
    A[l * K + k] = S[t];
  }
}

// In-place Gauss-Jordan inversion without pivoting (A_1 is SPD), step k:
// save row k and column k, then update every entry from the saved copies.
__global__ __launch_bounds__(kBlock) void k_gj_save(const double* A, int K, int k, double* row, double* col,
                                                    double* piv) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < K) {
    row[i] = A[size_t(k) * K + i];
    col[i] = A[size_t(i) * K + k];
  }
  if (i == 0) piv[k] = A[size_t(k) * K + k];
}
__global__ __launch_bounds__(kBlock) void k_gj_update(double* A, int K, int k, const double* row,
                                                      const double* col) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= int64_t(K) * K) return;
  const int i = int(t / K), j = int(t % K);
  const double p = row[k];
  const double rj = (j == k) ? 1.0 : row[j];
  if (i == k) {
    A[t] = rj / p;
  } else {
    const double aij = (j == k) ? 0.0 : A[t];
    A[t] = aij - col[i] * rj / p;
  }
}
__global__ __launch_bounds__(kBlock) void k_symmetrize(double* A, int K) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= int64_t(K) * K) return;
  const int i = int(t / K), j = int(t % K);
  if (i < j) {
    const double v = 0.5 * (A[t] + A[size_t(j) * K + i]);
    A[t] = v;
    A[size_t(j) * K + i] = v;
  }
}

// out = base + s * A v for a dense K x K matrix, one wavefront per row, FP64
// arithmetic whatever the I/O types (base may be null).
template <typename TB, typename TV, typename TO>
__global__ __launch_bounds__(kBlock) void k_gemv(const double* A, int K, const TB* base, double s, const TV* v,
                                                 TO* out) {
  const int row = (blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= K) return;
  double acc = 0.0;
  for (int j = lane; j < K; j += 64) acc += A[size_t(row) * K + j] * double(v[j]);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) out[row] = TO((base ? double(base[row]) : 0.0) + s * acc);
}

// ---------------------------------------------------------------------------
// Assembled operator of a coarse level as a 7^D-point stencil.
//
// On level g every cell's data Gram block is a linear function of the cell's
// polynomial moments M[c][e] = sum_i prod_p u_ip^e_p (u = level-g position
// in the cell minus 1/2, e_p = 0..6), so the data part of A_g[k, k+o] is
//   sum_c sum_e M[c][e] prod_p C[e_p][k_p - c_p][k_p + o_p - c_p]
// with the 7x4x4 table C of u^e coefficients of b_a(u+1/2) b_a'(u+1/2).
// Per dimension this is one and the same (7J) x (7N) matrix W acting on the
// axis (c_p, e_p), so the whole stencil is (W x ... x W) M: D banded passes
// (the Kronecker matvec of Alg. 2). lambda Lambda_g is added from the banded
// 1D factors; the result is stored offset-major, S[o][k].

// Moments of level g from the points, in the axis-interleaved layout
// index = sum_p (c_p * 7 + e_p) * (7 N_g)^(D-1-p) (mom zeroed first).
// Block (x, y, z): exponent tuples (e_1..e_{D-1}) starting at x * NR, level-g
// cells y, y + gridDim.y, ..., and the z-th of gridDim.z chunks of each
// cell's points. Threads are (tuple, stream): the NS = kBlock / NR streams
// take every NS-th point of a staged tile and are summed in LDS; a block
// stores its sums, or adds them atomically when a cell is split over
// gridDim.z > 1 blocks.
template <int D>
__global__ __launch_bounds__(kBlock) void k_level_moments(const double* t64, const uint32_t* cell,
                                                          const int32_t* off, int64_t n, int G, int g,
                                                          double* mom) {
  constexpr int E = 7;
  constexpr int TILE = 64;
  constexpr int NREST = (D == 1) ? 1 : (D == 2 ? 7 : (D == 3 ? 49 : (D == 4 ? 343 : 2401)));
  constexpr int NR = NREST < kBlock ? NREST : kBlock;   // tuples per block
  constexpr int NS = kBlock / NR;                       // point streams per tuple
  __shared__ double pw[TILE][D][E];
  __shared__ double red[kBlock][E];   // per-thread sums of a cell, reduced over the streams
  const int sh = G - g;
  const int S = D * sh;
  const uint32_t ncells = 1u << (D * g);
  const int tup = threadIdx.x % NR, strm = threadIdx.x / NR;
  const int r = blockIdx.x * NR + tup;
  const bool active = r < NREST && strm < NS;
  int er[D];
  {
    int rem = r;
#pragma unroll
    for (int p = D - 1; p >= 1; --p) { er[p] = rem % E; rem /= E; }
    er[0] = 0;
  }
  const uint32_t maskN = (1u << G) - 1u, maskSh = (1u << sh) - 1u;
  const double scale = 1.0 / double(1u << sh);
  for (uint32_t cidx = blockIdx.y; cidx < ncells; cidx += gridDim.y) {
    const int64_t c0 = off[size_t(cidx) << S], c1 = off[size_t(cidx + 1) << S];
    const int64_t per = (c1 - c0 + gridDim.z - 1) / gridDim.z;
    const int64_t b0 = c0 + int64_t(blockIdx.z) * per;
    const int64_t b1 = min(c1, b0 + per);
    double acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
    for (int64_t base = b0; base < b1; base += TILE) {
      __syncthreads();   // previous readers of pw are done
      for (int w = threadIdx.x; w < TILE * D; w += kBlock) {
        const int pt = w / D, p = w % D;
        const int64_t i = base + pt;
        double u = 0.0;
        const bool ok = i < b1;
        if (ok) {
          const uint32_t cfp = (cell[i] >> (G * (D - 1 - p))) & maskN;
          u = (double(cfp & maskSh) + t64[size_t(p) * n + i]) * scale - 0.5;
        }
        double v = ok ? 1.0 : 0.0;
        for (int e = 0; e < E; ++e) { pw[pt][p][e] = v; v *= u; }
      }
      __syncthreads();
      if (active) {
        const int cnt = int(min(int64_t(TILE), b1 - base));
        for (int pt = strm; pt < cnt; pt += NS) {
          double prod = 1.0;
#pragma unroll
          for (int p = 1; p < D; ++p) prod *= pw[pt][p][er[p]];
#pragma unroll
          for (int e = 0; e < E; ++e) acc[e] += prod * pw[pt][0][e];
        }
      }
    }
    if (b0 < b1) {   // uniform in the block
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) red[threadIdx.x][e] = acc[e];
      }
      __syncthreads();
      int cc[D];
      morton_decode<D>(cidx, g, cc);
      const int64_t A = int64_t(E) << g;   // 7 N_g
      for (int w = threadIdx.x; w < NR * E; w += kBlock) {
        const int tu = w / E, e = w % E;
        const int rr = blockIdx.x * NR + tu;
        if (rr >= NREST) continue;
        double sum = 0.0;
        for (int st = 0; st < NS; ++st) sum += red[st * NR + tu][e];
        int64_t idx = int64_t(cc[0]) * E + e;
        int rem = rr, ep[D];
#pragma unroll
        for (int p = D - 1; p >= 1; --p) { ep[p] = rem % E; rem /= E; }
#pragma unroll
        for (int p = 1; p < D; ++p) idx = idx * A + (int64_t(cc[p]) * E + ep[p]);
        if (gridDim.z > 1) atomicAdd(&mom[idx], sum);
        else mom[idx] = sum;
      }
      __syncthreads();   // red is free again
    }
  }
}

// Moments of the level g-1 cells from those of their children on level g,
// along one dimension (D passes give all of them): with centred coordinates
// u in a parent cell and u' in its child b (0: lower half, 1: upper half),
// u = u'/2 + (2b-1)/4, so u^e = sum_{j<=e} C(e,j) 2^-j ((2b-1)/4)^(e-j) u'^j.
// in: [outer][7 * 2Nc][inner], out: [outer][7 * Nc][inner], same axis
// interleaving as k_level_moments.
__global__ __launch_bounds__(kBlock) void k_moments_coarsen(const double* in, double* out, int Nc, int64_t outer,
                                                            int64_t inner) {
  constexpr int E = 7;
  const int64_t total = outer * E * Nc * inner;
  for (int64_t idx = int64_t(blockIdx.x) * kBlock + threadIdx.x; idx < total; idx += int64_t(gridDim.x) * kBlock) {
    const int64_t i = idx % inner;
    int64_t t = idx / inner;
    const int e = int(t % E);
    t /= E;
    const int64_t C = t % Nc;
    const int64_t o = t / Nc;
    double sum = 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double sb = b ? 0.25 : -0.25;
      const double* src = in + ((o * 2 * Nc + 2 * C + b) * E) * inner + i;
      double coef = ldexp(1.0, -e);   // C(e,j) 2^-j, exact
      double shift = 1.0;             // sb^(e-j)
      for (int j = e; j >= 0; --j) {
        sum += coef * shift * src[int64_t(j) * inner];
        coef = coef * 2.0 * j / double(e - j + 1);
        shift *= sb;
      }
    }
    out[idx] = sum;
  }
}

// One Kronecker pass: axis p goes from (c, e) (size 7N) to (k, o+3) (size 7J).
// in [outer][7N][inner] -> out [outer][7J][inner].
__global__ __launch_bounds__(kBlock) void k_stencil_pass(const double* in, double* out, const double* ctab,
                                                         int N, int64_t inner, int64_t total) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= total) return;
  const int J = N + kDeg;
  const int64_t ii = t % inner;
  const int64_t rest = t / inner;
  const int ko = int(rest % (7 * J));
  const int64_t outer = rest / (7 * J);
  const int k = ko / 7, o = ko % 7 - 3;
  const int l = k + o;
  double sacc = 0.0;
  if (l >= 0 && l < J) {
    const int clo = max(0, max(k, l) - 3), chi = min(N - 1, min(k, l));
    const int64_t ibase = outer * (int64_t(7) * N) * inner + ii;
    for (int c = clo; c <= chi; ++c) {
      const int pi = (k - c) * 4 + (l - c);
#pragma unroll
      for (int e = 0; e < 7; ++e) sacc += ctab[e * 16 + pi] * in[ibase + (int64_t(c) * 7 + e) * inner];
    }
  }
  out[t] = sacc;
}

// S[h][k] = (data stencil in the interleaved layout) + lambda Lambda_g[k, k+o]
// for the offsets o = NO/2 + h, h = 0..NO/2 (the centre and the offsets after
// it in the base-7 order, i.e. the flat offset is >= 0): A_g is symmetric, so
// the other half is A[k][k-o] = S[h][k-o]. Entries whose neighbour falls
// outside the grid are zero.
template <int D>
__global__ __launch_bounds__(kBlock) void k_stencil_finalize(const double* inter, const double* band, int J,
                                                             int64_t K, double lam, double* S64, float* S32) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  int NO = 1;
#pragma unroll
  for (int p = 0; p < D; ++p) NO *= 7;
  if (t >= int64_t((NO + 1) / 2) * K) return;
  const int oidx = NO / 2 + int(t / K);
  const int64_t k = t % K;
  int kp[D], op[D];
  {
    int64_t rk = k;
    int ro = oidx;
#pragma unroll
    for (int p = D - 1; p >= 0; --p) {
      kp[p] = int(rk % J); rk /= J;
      op[p] = ro % 7; ro /= 7;
    }
  }
  bool inside = true;
  int64_t ii = 0;
#pragma unroll
  for (int p = 0; p < D; ++p) {
    const int l = kp[p] + op[p] - 3;
    inside = inside && l >= 0 && l < J;
    ii = ii * (int64_t(7) * J) + (int64_t(kp[p]) * 7 + op[p]);
  }
  double v = 0.0;
  if (inside) {
    double mv[D], g1v[D], g2v[D];
#pragma unroll
    for (int p = 0; p < D; ++p) {
      const double* bp = band + size_t(p) * 3 * J * 7;
      mv[p] = bp[size_t(kp[p]) * 7 + op[p]];
      g1v[p] = bp[size_t(J) * 7 + size_t(kp[p]) * 7 + op[p]];
      g2v[p] = bp[size_t(2 * J) * 7 + size_t(kp[p]) * 7 + op[p]];
    }
    double lm = 0.0;
#pragma unroll
    for (int p = 0; p < D; ++p) {
      double w = g2v[p];
#pragma unroll
      for (int q = 0; q < D; ++q)
        if (q != p) w *= mv[q];
      lm += w;
    }
#pragma unroll
    for (int p = 0; p < D; ++p)
#pragma unroll
      for (int q = p + 1; q < D; ++q) {
        double w = 2.0 * g1v[p] * g1v[q];
#pragma unroll
        for (int r = 0; r < D; ++r)
          if (r != p && r != q) w *= mv[r];
        lm += w;
      }
    v = inter[ii] + lam * lm;
  }
  S64[t] = v;
  S32[t] = float(v);
}

// v = A_g x with the stored half stencil (k_stencil_finalize):
//   v[k] = S[0][k] x[k] + sum_{h>=1} (S[h][k] x[k + off[h]] + S[h][k - off[h]] x[k - off[h]]),
// the last term being A[k][k-off] = A[k-off][k]; then the epilogue: out = v
// (kStPlain), out = x + w (b - v) (kStJacobi, one damped Jacobi sweep of
// Alg. 6; out must not alias x), or out = v - b (kStResidual). A neighbour
// outside the grid has S = 0 (its index is clamped into range, so the finite
// value read there is multiplied by zero); a mirrored row index below zero is
// skipped.
enum StencilEpilogue : int { kStPlain = 0, kStJacobi = 1, kStResidual = 2, kStJacobiZero = 3 };
constexpr int kStRows = kBlock / 7;   // 36 rows per block

template <int D>
constexpr int stencil_half() {
  int no = 1;
  for (int p = 0; p < D; ++p) no *= 7;
  return (no + 1) / 2;
}

// Input value at flat index i: x[i], or for kStJacobiZero the first sweep
// from zero, w[i] b[i] (x is not read).
template <typename T, int EPI>
__device__ __forceinline__ T stencil_in(const T* x, const T* b, const T* w, int64_t i) {
  if constexpr (EPI == kStJacobiZero) return w[i] * b[i];
  else return x[i];
}

template <typename T, int EPI>
__device__ __forceinline__ void stencil_out(const T* x, T* out, const T* b, const T* w, int64_t k, T v) {
  if constexpr (EPI == kStPlain) out[k] = v;
  else if constexpr (EPI == kStJacobi) out[k] = x[k] + w[k] * (b[k] - v);
  else if constexpr (EPI == kStResidual) out[k] = v - b[k];
  else {
    const T x1 = w[k] * b[k];
    out[k] = x1 + w[k] * (b[k] - v);
  }
}

// Flat index offset (>= 0) of stored stencil point h: the base-7 digits of
// NO/2 + h, each minus 3, weighted by the strides J^(D-1-p).
template <int D>
__device__ __forceinline__ int64_t stencil_off(int h, int J) {
  int o = stencil_half<D>() - 1 + h;
  int64_t off = 0, stride = 1;
#pragma unroll
  for (int p = D - 1; p >= 0; --p) {
    off += int64_t(o % 7 - 3) * stride;
    o /= 7;
    stride *= J;
  }
  return off;
}

// Stored offsets h and their mirrors, for row k.
template <typename T, int D, int EPI>
__device__ __forceinline__ void stencil_pair(const T* S, int J, const T* x, const T* b, const T* w, int64_t K,
                                             int64_t k, int h, T& a0, T& a1) {
  const int64_t off = stencil_off<D>(h, J);
  int64_t i = k + off;
  i = i >= K ? K - 1 : i;
  a0 += S[int64_t(h) * K + k] * stencil_in<T, EPI>(x, b, w, i);
  const int64_t j = k - off;
  if (h > 0 && j >= 0) a1 += S[int64_t(h) * K + j] * stencil_in<T, EPI>(x, b, w, j);
}

// Rows k of the level in blocks of 36; the stored offsets are dealt to 7
// groups of threads per row and the group sums are added in LDS. For levels
// with many rows (streams the stored half once; its mirror reads come back
// from cache).
template <typename T, int D, int EPI>
__global__ __launch_bounds__(kBlock) void k_stencil_apply(const T* S, int J, const T* x, T* out, const T* b,
                                                          const T* w, int64_t K) {
  constexpr int NH = stencil_half<D>();
  constexpr int PERG = (NH + 6) / 7;
  __shared__ T part[7][kStRows];
  const int grp = threadIdx.x / kStRows;
  const int rl = threadIdx.x % kStRows;
  // contiguous row ranges per XCD: a stored entry and its mirrored read meet in one L2
  const int64_t k = int64_t(xcd_block()) * kStRows + rl;
  if (grp < 7) {
    T a0 = T(0), a1 = T(0);
    if (k < K) {
      const int h1 = min(NH, (grp + 1) * PERG);
      for (int h = grp * PERG; h < h1; ++h) stencil_pair<T, D, EPI>(S, J, x, b, w, K, k, h, a0, a1);
    }
    part[grp][rl] = a0 + a1;
  }
  __syncthreads();
  if (threadIdx.x < kStRows && k < K) {
    T v = T(0);
#pragma unroll
    for (int q = 0; q < 7; ++q) v += part[q][threadIdx.x];
    stencil_out<T, EPI>(x, out, b, w, k, v);
  }
}

// The same product for levels with few rows, where the kernel above is
// latency-bound: 8 rows per block, 32 threads per row, each taking every
// 32nd stored offset; a row's 8 threads in a wave are summed by lane
// exchanges, the 4 waves in LDS.
constexpr int kStSmallRows = 8;
constexpr int kStSmallCols = kBlock / kStSmallRows;
constexpr int64_t kStSmallMaxK = 16384;

template <typename T, int D, int EPI>
__global__ __launch_bounds__(kBlock) void k_stencil_apply_small(const T* S, int J, const T* x, T* out, const T* b,
                                                                const T* w, int64_t K) {
  constexpr int NH = stencil_half<D>();
  constexpr int PER = (NH + kStSmallCols - 1) / kStSmallCols;
  static_assert(kStSmallRows == 8 && kBlock == 256, "lane layout below");
  __shared__ T part[kBlock / 64][kStSmallRows];
  const int r = threadIdx.x % kStSmallRows;
  const int c = threadIdx.x / kStSmallRows;
  const int64_t k = int64_t(blockIdx.x) * kStSmallRows + r;
  T a0 = T(0), a1 = T(0);
  if (k < K) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int h = c + q * kStSmallCols;
      if (h < NH) stencil_pair<T, D, EPI>(S, J, x, b, w, K, k, h, a0, a1);
    }
  }
  // lanes r, r + 8, ..., r + 56 of a wave hold row r
  T a = a0 + a1;
  a += __shfl_xor(a, 8);
  a += __shfl_xor(a, 16);
  a += __shfl_xor(a, 32);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  if (lane < kStSmallRows) part[wv][lane] = a;
  __syncthreads();
  if (threadIdx.x < kStSmallRows && k < K) {
    T v = part[0][r];
#pragma unroll
    for (int q = 1; q < kBlock / 64; ++q) v += part[q][r];
    stencil_out<T, EPI>(x, out, b, w, k, v);
  }
}

// One colour class of the SSOR sweep (Sec. 3.2.2) on a stencil level: the
// rows k whose multi-index has j_p = c_p (mod 4) in every dimension, c the
// class's base-4 digits in C order. Two rows of a class are at least four
// apart in some dimension, outside each other's 7^d stencil, so the class is
// updated at once and in place:
//   x_k <- x_k + omega (b_k - (A x)_k) / A_kk.
// Same row layout as k_stencil_apply_small (8 rows per block, 32 threads per
// row); every read of x in a block precedes the barrier, every write follows it.
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_stencil_color(const T* S, int J, T* x, const T* b, T omega, int color,
                                                          int64_t rows, int64_t K) {
  constexpr int NH = stencil_half<D>();
  constexpr int PER = (NH + kStSmallCols - 1) / kStSmallCols;
  __shared__ T part[kBlock / 64][kStSmallRows];
  const int r = threadIdx.x % kStSmallRows;
  const int c = threadIdx.x / kStSmallRows;
  const int64_t q = int64_t(blockIdx.x) * kStSmallRows + r;   // row of the class
  int64_t k = -1;
  if (q < rows) {
    int64_t rem = q, kk = 0, stride = 1;
    int col = color;
#pragma unroll
    for (int p = D - 1; p >= 0; --p) {
      const int cp = col % 4;
      col /= 4;
      const int64_t m = (J - cp + 3) / 4;
      const int64_t ip = rem % m;
      rem /= m;
      kk += (cp + 4 * ip) * stride;
      stride *= J;
    }
    k = kk;
  }
  T a0 = T(0), a1 = T(0);
  if (k >= 0) {
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int h = c + s * kStSmallCols;
      if (h < NH) stencil_pair<T, D, kStPlain>(S, J, x, nullptr, nullptr, K, k, h, a0, a1);
    }
  }
  T a = a0 + a1;
  a += __shfl_xor(a, 8);
  a += __shfl_xor(a, 16);
  a += __shfl_xor(a, 32);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  if (lane < kStSmallRows) part[wv][lane] = a;
  __syncthreads();
  if (threadIdx.x < kStSmallRows && k >= 0) {
    T v = part[0][r];
#pragma unroll
    for (int s = 1; s < kBlock / 64; ++s) v += part[s][r];
    x[k] = x[k] + omega * (b[k] - v) / S[k];
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
static inline unsigned blocks_for(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

template <int D, typename T, int MODE, int TBF, bool WL, bool DET = false>
static hipError_t launch_data_tb(const DataArgs& a, hipStream_t st) {
  const int Tg = 1 << a.tb;
  int patch = 1;
  for (int p = 0; p < D; ++p) patch *= (Tg + kDeg);
  const size_t lds = data_lds<D, T, MODE, Group<D>::STAGE_C, WL, DET>(patch, a.ppb, Group<D>::Q).total;
  if (a.ppb > Group<D>::PPB) return hipErrorInvalidValue;
  const unsigned grid = WL ? unsigned(a.wl_groups) : unsigned((a.n + a.ppb - 1) / a.ppb);
  if (grid == 0) return hipSuccess;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_data<D, T, MODE, TBF, WL, DET>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_data<D, T, MODE, TBF, WL, DET>), dim3(grid), dim3(kBlock), lds, st, a);
  if constexpr (DET) {
    int64_t K = 1;
    for (int p = 0; p < D; ++p) K *= (1 << a.g) + kDeg;
    hipLaunchKernelGGL((k_det_reduce<D, T>), dim3(unsigned((K + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       a.det_part, a.det_tile_first, static_cast<T*>(a.out), a.g, a.tb, K);
  }
  return hipGetLastError();
}

template <int D, typename T, int MODE>
static hipError_t launch_data_d(const DataArgs& a, hipStream_t st) {
  if (a.det) {
    if (!a.wl_items || !a.det_part || !a.det_tile_first) return hipErrorInvalidValue;
    if (a.tb == kTileBits[D]) return launch_data_tb<D, T, MODE, kTileBits[D], true, true>(a, st);
    return launch_data_tb<D, T, MODE, -1, true, true>(a, st);
  }
  if constexpr (MODE == kApply) {
    if (a.wl_items) {
      if (a.tb == kTileBits[D]) return launch_data_tb<D, T, MODE, kTileBits[D], true>(a, st);
      return launch_data_tb<D, T, MODE, -1, true>(a, st);
    }
  }
  if (a.tb == kTileBits[D]) return launch_data_tb<D, T, MODE, kTileBits[D], false>(a, st);
  return launch_data_tb<D, T, MODE, -1, false>(a, st);
}


template <typename T, int MODE>
static hipError_t launch_data_t(int D, const DataArgs& a, hipStream_t st) {
  switch (D) {
    case 1: return launch_data_d<1, T, MODE>(a, st);
    case 2: return launch_data_d<2, T, MODE>(a, st);
    case 3: return launch_data_d<3, T, MODE>(a, st);
    case 4: return launch_data_d<4, T, MODE>(a, st);
    case 5: return launch_data_d<5, T, MODE>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_data(int D, bool fp32, int mode, const DataArgs& a, hipStream_t st) {
  if (fp32) {
    if (mode == kApply) return launch_data_t<float, kApply>(D, a, st);
    return hipErrorInvalidValue;
  }
  if (mode == kApply) return launch_data_t<double, kApply>(D, a, st);
  if (mode == kRhs) return launch_data_t<double, kRhs>(D, a, st);
  if (mode == kDiag) return launch_data_t<double, kDiag>(D, a, st);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_lambda_pass(const LambdaArgs<T>& a, hipStream_t st) {
  if (a.K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lambda_pass<T>, dim3(blocks_for(a.K)), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_lambda_fused(int D, const T* c, T* out, const T* band, int J, T lam, hipStream_t st) {
  if (D == 3) {
    const int nt = (J + kLamB - 1) / kLamB, B = (J + nt - 1) / nt;   // B <= kLamB
    const int nt0 = (J + kLamC0 - 1) / kLamC0;
    hipLaunchKernelGGL((k_lambda_fused3<T, false, kLamC0>), dim3(unsigned(nt0 * nt * nt)), dim3(kBlock), 0, st, c,
                       nullptr, nullptr, out, band, J, B, nt, nt0, lam);
    return hipGetLastError();
  }
  if (D == 2) {
    const int nt0 = (J + kLam2B0 - 1) / kLam2B0, nt1 = (J + kLam2B1 - 1) / kLam2B1;
    const int B0 = (J + nt0 - 1) / nt0, B1 = (J + nt1 - 1) / nt1;
    hipLaunchKernelGGL(k_lambda_fused2<T>, dim3(unsigned(nt0 * nt1)), dim3(kBlock), 0, st, c, out, band, J, B0, B1,
                       nt1, lam);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
template <typename T>
hipError_t launch_lambda_tail3(const T* t0, const T* t1, const T* t2, T* out, const T* band, int J, int64_t outer,
                               T lam, hipStream_t st) {
  const int nt = (J + kLamB - 1) / kLamB, B = (J + nt - 1) / nt;
  const int nt0 = (J + kLamC0x3 - 1) / kLamC0x3;
  const int64_t blocks = outer * nt0 * nt * nt;
  if (blocks == 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_lambda_fused3<T, true, kLamC0x3>), dim3(unsigned(blocks)), dim3(kBlock), 0, st, t0, t1, t2,
                     out, band, J, B, nt, nt0, lam);
  return hipGetLastError();
}
template hipError_t launch_lambda_tail3<double>(const double*, const double*, const double*, double*, const double*,
                                                int, int64_t, double, hipStream_t);
template hipError_t launch_lambda_tail3<float>(const float*, const float*, const float*, float*, const float*, int,
                                               int64_t, float, hipStream_t);
template hipError_t launch_lambda_fused<double>(int, const double*, double*, const double*, int, double, hipStream_t);
template hipError_t launch_lambda_fused<float>(int, const float*, float*, const float*, int, float, hipStream_t);

template hipError_t launch_lambda_pass<double>(const LambdaArgs<double>&, hipStream_t);
template hipError_t launch_lambda_pass<float>(const LambdaArgs<float>&, hipStream_t);

hipError_t launch_lambda_diag(int D, const double* band, int J, int64_t K, double lam, double* out,
                              hipStream_t st) {
  const unsigned g = blocks_for(K);
  switch (D) {
    case 1: hipLaunchKernelGGL(k_lambda_diag<1>, dim3(g), dim3(kBlock), 0, st, band, J, K, lam, out); break;
    case 2: hipLaunchKernelGGL(k_lambda_diag<2>, dim3(g), dim3(kBlock), 0, st, band, J, K, lam, out); break;
    case 3: hipLaunchKernelGGL(k_lambda_diag<3>, dim3(g), dim3(kBlock), 0, st, band, J, K, lam, out); break;
    case 4: hipLaunchKernelGGL(k_lambda_diag<4>, dim3(g), dim3(kBlock), 0, st, band, J, K, lam, out); break;
    case 5: hipLaunchKernelGGL(k_lambda_diag<5>, dim3(g), dim3(kBlock), 0, st, band, J, K, lam, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transfer(bool prolong, const TransferArgs<T>& a, hipStream_t st) {
  if (a.Kout == 0) return hipSuccess;
  if (prolong) hipLaunchKernelGGL(k_prolong_pass<T>, dim3(blocks_for(a.Kout)), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL(k_restrict_pass<T>, dim3(blocks_for(a.Kout)), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_transfer<double>(bool, const TransferArgs<double>&, hipStream_t);
template hipError_t launch_transfer<float>(bool, const TransferArgs<float>&, hipStream_t);

template <typename T, int D>
static hipError_t launch_transfer_fused_d(bool prolong, const T* in, const T* sub, T* out, int Jc, int Jf,
                                          int subtract, const T* wj, T* aj, hipStream_t st) {
  int64_t Kc = 1, Kf = 1;
  for (int p = 0; p < D; ++p) { Kc *= Jc; Kf *= Jf; }
  if (prolong) {
    hipLaunchKernelGGL((k_prolong_fused<D, T>), dim3(blocks_for(Kf)), dim3(kBlock), 0, st, in, out, Jc, Jf, Kf,
                       subtract);
  } else if constexpr (D <= 4) {
    const int per_block = kBlock / kRestrictLanes;
    hipLaunchKernelGGL((k_restrict_fused<D, T>), dim3(unsigned((Kc + per_block - 1) / per_block)), dim3(kBlock), 0,
                       st, in, sub, out, Jc, Jf, Kc, wj, aj);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transfer_fused(int D, bool prolong, const T* in, const T* sub, T* out, int Jc, int Jf,
                                 int subtract, const T* wj, T* aj, hipStream_t st) {
  switch (D) {
    case 1: return launch_transfer_fused_d<T, 1>(prolong, in, sub, out, Jc, Jf, subtract, wj, aj, st);
    case 2: return launch_transfer_fused_d<T, 2>(prolong, in, sub, out, Jc, Jf, subtract, wj, aj, st);
    case 3: return launch_transfer_fused_d<T, 3>(prolong, in, sub, out, Jc, Jf, subtract, wj, aj, st);
    case 4: return launch_transfer_fused_d<T, 4>(prolong, in, sub, out, Jc, Jf, subtract, wj, aj, st);
    case 5:
      if (!prolong) return hipErrorInvalidValue;   // restriction at d = 5 runs pass by pass
      return launch_transfer_fused_d<T, 5>(prolong, in, sub, out, Jc, Jf, subtract, wj, aj, st);
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_transfer_fused<double>(int, bool, const double*, const double*, double*, int, int, int,
                                                  const double*, double*, hipStream_t);
template hipError_t launch_transfer_fused<float>(int, bool, const float*, const float*, float*, int, int, int,
                                                 const float*, float*, hipStream_t);

template <typename T>
hipError_t launch_jacobi_first(T* alpha, const T* wdinv, const T* b, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_first<T>, dim3(blocks_for(K)), dim3(kBlock), 0, st, alpha, wdinv, b, K);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_jacobi(T* alpha, const T* wdinv, const T* b, const T* Ax, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi<T>, dim3(blocks_for(K)), dim3(kBlock), 0, st, alpha, wdinv, b, Ax, K);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_residual(T* r, const T* Ax, const T* b, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_residual<T>, dim3(blocks_for(K)), dim3(kBlock), 0, st, r, Ax, b, K);
  return hipGetLastError();
}
template hipError_t launch_jacobi_first<double>(double*, const double*, const double*, int64_t, hipStream_t);
template hipError_t launch_jacobi_first<float>(float*, const float*, const float*, int64_t, hipStream_t);
template hipError_t launch_jacobi<double>(double*, const double*, const double*, const double*, int64_t, hipStream_t);
template hipError_t launch_jacobi<float>(float*, const float*, const float*, const float*, int64_t, hipStream_t);
template hipError_t launch_residual<double>(double*, const double*, const double*, int64_t, hipStream_t);
template hipError_t launch_residual<float>(float*, const float*, const float*, int64_t, hipStream_t);

static inline unsigned reduce_blocks(int64_t K) {
  int64_t b = (K + kBlock * 4 - 1) / (kBlock * 4);
  if (b < 1) b = 1;
  if (b > kMaxPartials) b = kMaxPartials;
  return unsigned(b);
}

template <typename TX, typename TY>
hipError_t launch_dot(const TX* x, const TY* y, int64_t K, double* partial, double* slot, hipStream_t st) {
  const unsigned nb = reduce_blocks(K);
  hipLaunchKernelGGL((k_dot_partial<TX, TY>), dim3(nb), dim3(kBlock), 0, st, x, y, K, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, st, partial, int(nb), slot);
  return hipGetLastError();
}

template <typename TX, typename TY>
hipError_t launch_dot_partial(const TX* x, const TY* y, int64_t K, double* partial, int* nb, hipStream_t st) {
  const unsigned b = reduce_blocks(K);
  hipLaunchKernelGGL((k_dot_partial<TX, TY>), dim3(b), dim3(kBlock), 0, st, x, y, K, partial);
  *nb = int(b);
  return hipGetLastError();
}
template hipError_t launch_dot_partial<double, double>(const double*, const double*, int64_t, double*, int*,
                                                       hipStream_t);

hipError_t launch_cg_step_norms(double* alpha, double* r, const double* p, const double* v, const double* z,
                                int64_t K, const double* num, double* den, double* partial, double* rr,
                                double* rz, const double* wz, double* zf, const double* den_part, int den_nb,
                                hipStream_t st) {
  const unsigned nb = reduce_blocks(K);
  hipLaunchKernelGGL(k_cg_step_norms, dim3(nb), dim3(kBlock), 0, st, alpha, r, p, v, z, K, num, den, partial, wz,
                     zf, den_part, den_nb);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kBlock), 0, st, partial, int(nb), z ? 2 : 1, rr, rz);
  return hipGetLastError();
}
template hipError_t launch_dot<double, double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template hipError_t launch_dot<float, float>(const float*, const float*, int64_t, double*, double*, hipStream_t);

template <typename TA, typename T>
hipError_t launch_cg_step(TA* alpha, T* r, const T* p, const T* v, int64_t K, const double* num,
                          const double* den, hipStream_t st) {
  hipLaunchKernelGGL((k_cg_step<TA, T>), dim3(blocks_for(K)), dim3(kBlock), 0, st, alpha, r, p, v, K, num, den);
  return hipGetLastError();
}
template hipError_t launch_cg_step<double, double>(double*, double*, const double*, const double*, int64_t,
                                                   const double*, const double*, hipStream_t);
template hipError_t launch_cg_step<float, float>(float*, float*, const float*, const float*, int64_t,
                                                 const double*, const double*, hipStream_t);

template <typename T>
hipError_t launch_p_update(T* p, const T* z, int64_t K, const double* num, const double* den, hipStream_t st) {
  hipLaunchKernelGGL(k_p_update<T>, dim3(blocks_for(K)), dim3(kBlock), 0, st, p, z, K, num, den);
  return hipGetLastError();
}
template hipError_t launch_p_update<double>(double*, const double*, int64_t, const double*, const double*, hipStream_t);
template hipError_t launch_p_update<float>(float*, const float*, int64_t, const double*, const double*, hipStream_t);

hipError_t launch_p_update_sum(double* p, const double* z, int64_t K, double* num, const double* num_part, int nb,
                               const double* sub, const double* den, hipStream_t st) {
  hipLaunchKernelGGL(k_p_update_sum, dim3(blocks_for(K)), dim3(kBlock), 0, st, p, z, K, num, num_part, nb, sub, den);
  return hipGetLastError();
}

hipError_t launch_scale_mul(const float* x, double* y, int64_t K, const double* smul, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_mul<float, double>), dim3(blocks_for(K)), dim3(kBlock), 0, st, x, y, K, smul);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_scale_copy(const TI* x, TO* y, int64_t K, double scale, const double* sden, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_copy<TI, TO>), dim3(blocks_for(K)), dim3(kBlock), 0, st, x, y, K, scale, sden);
  return hipGetLastError();
}
template hipError_t launch_scale_copy<double, float>(const double*, float*, int64_t, double, const double*, hipStream_t);
template hipError_t launch_scale_copy<float, double>(const float*, double*, int64_t, double, const double*, hipStream_t);
template hipError_t launch_scale_copy<double, double>(const double*, double*, int64_t, double, const double*, hipStream_t);
template hipError_t launch_scale_copy<float, float>(const float*, float*, int64_t, double, const double*, hipStream_t);

template <typename TI, typename TO>
hipError_t launch_axpy_conv(const TI* x, TO* y, int64_t K, double scale, const double* smul, hipStream_t st) {
  hipLaunchKernelGGL((k_axpy_conv<TI, TO>), dim3(blocks_for(K)), dim3(kBlock), 0, st, x, y, K, scale, smul);
  return hipGetLastError();
}
template hipError_t launch_axpy_conv<float, double>(const float*, double*, int64_t, double, const double*, hipStream_t);

hipError_t launch_mul(const double* d, const double* x, double* y, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_mul, dim3(blocks_for(K)), dim3(kBlock), 0, st, d, x, y, K);
  return hipGetLastError();
}
hipError_t launch_lanczos_w(const double* d, const double* Ax, const double* vprev, const double* b2prev, double* w,
                            int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_lanczos_w, dim3(blocks_for(K)), dim3(kBlock), 0, st, d, Ax, vprev, b2prev, w, K);
  return hipGetLastError();
}
hipError_t launch_axpy(double scale, const double* s, const double* x, double* y, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(K)), dim3(kBlock), 0, st, scale, s, x, y, K);
  return hipGetLastError();
}
hipError_t launch_start_vector(double* u, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_start_vector, dim3(blocks_for(K)), dim3(kBlock), 0, st, u, K);
  return hipGetLastError();
}
hipError_t launch_rsqrt_vec(const double* D, double* out, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_rsqrt_vec, dim3(blocks_for(K)), dim3(kBlock), 0, st, D, out, K);
  return hipGetLastError();
}
hipError_t launch_wdinv(const double* D, double omega, double* w64, float* w32, int64_t K, hipStream_t st) {
  hipLaunchKernelGGL(k_wdinv, dim3(blocks_for(K)), dim3(kBlock), 0, st, D, omega, w64, w32, K);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(T* x, T v, int64_t K, hipStream_t st) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(K)), dim3(kBlock), 0, st, x, v, K);
  return hipGetLastError();
}
template hipError_t launch_fill<double>(double*, double, int64_t, hipStream_t);
template hipError_t launch_fill<float>(float*, float, int64_t, hipStream_t);
template hipError_t launch_fill<int>(int*, int, int64_t, hipStream_t);

hipError_t launch_check_finite(const double* x, int64_t K, int* flag, hipStream_t st) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(K)), dim3(kBlock), 0, st, x, K, flag);
  return hipGetLastError();
}

hipError_t launch_bin(int D, const double* x, int64_t n, const BoxArgs& box, uint32_t* key, uint32_t* idx,
                      int* flag, hipStream_t st) {
  const unsigned g = blocks_for(n);
  switch (D) {
    case 1: hipLaunchKernelGGL(k_bin<1>, dim3(g), dim3(kBlock), 0, st, x, n, box, key, idx, flag); break;
    case 2: hipLaunchKernelGGL(k_bin<2>, dim3(g), dim3(kBlock), 0, st, x, n, box, key, idx, flag); break;
    case 3: hipLaunchKernelGGL(k_bin<3>, dim3(g), dim3(kBlock), 0, st, x, n, box, key, idx, flag); break;
    case 4: hipLaunchKernelGGL(k_bin<4>, dim3(g), dim3(kBlock), 0, st, x, n, box, key, idx, flag); break;
    case 5: hipLaunchKernelGGL(k_bin<5>, dim3(g), dim3(kBlock), 0, st, x, n, box, key, idx, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_place(int D, const double* x, const double* y, const uint32_t* idx, int64_t n,
                        const BoxArgs& box, double* t64, float* t32, uint32_t* cell, double* ys, hipStream_t st) {
  const unsigned g = blocks_for(n);
  switch (D) {
    case 1: hipLaunchKernelGGL(k_place<1>, dim3(g), dim3(kBlock), 0, st, x, y, idx, n, box, t64, t32, cell, ys); break;
    case 2: hipLaunchKernelGGL(k_place<2>, dim3(g), dim3(kBlock), 0, st, x, y, idx, n, box, t64, t32, cell, ys); break;
    case 3: hipLaunchKernelGGL(k_place<3>, dim3(g), dim3(kBlock), 0, st, x, y, idx, n, box, t64, t32, cell, ys); break;
    case 4: hipLaunchKernelGGL(k_place<4>, dim3(g), dim3(kBlock), 0, st, x, y, idx, n, box, t64, t32, cell, ys); break;
    case 5: hipLaunchKernelGGL(k_place<5>, dim3(g), dim3(kBlock), 0, st, x, y, idx, n, box, t64, t32, cell, ys); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_offsets(const uint32_t* key, int64_t n, int64_t ncells, int32_t* off, hipStream_t st) {
  hipLaunchKernelGGL(k_offsets, dim3(blocks_for(ncells + 1)), dim3(kBlock), 0, st, key, n, ncells, off);
  return hipGetLastError();
}

hipError_t launch_eval(int D, const double* alpha, const double* xq, int64_t m, const BoxArgs& box, double* yq,
                       hipStream_t st) {
  if (m == 0) return hipSuccess;
  const unsigned g = blocks_for(m);
  switch (D) {
    case 1: hipLaunchKernelGGL(k_eval<1>, dim3(g), dim3(kBlock), 0, st, alpha, xq, m, box, yq); break;
    case 2: hipLaunchKernelGGL(k_eval<2>, dim3(g), dim3(kBlock), 0, st, alpha, xq, m, box, yq); break;
    case 3: hipLaunchKernelGGL(k_eval<3>, dim3(g), dim3(kBlock), 0, st, alpha, xq, m, box, yq); break;
    case 4: hipLaunchKernelGGL(k_eval<4>, dim3(g), dim3(kBlock), 0, st, alpha, xq, m, box, yq); break;
    case 5: hipLaunchKernelGGL(k_eval<5>, dim3(g), dim3(kBlock), 0, st, alpha, xq, m, box, yq); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dense_from_stencil(int D, const double* S, int J, int64_t K, double* A, hipStream_t st) {
  int64_t NO = 1;
  for (int p = 0; p < D; ++p) NO *= 7;
  const unsigned g = blocks_for((NO + 1) / 2 * K);   // the stored half
  switch (D) {
    case 1: hipLaunchKernelGGL(k_dense_from_stencil<1>, dim3(g), dim3(kBlock), 0, st, S, J, K, A); break;
    case 2: hipLaunchKernelGGL(k_dense_from_stencil<2>, dim3(g), dim3(kBlock), 0, st, S, J, K, A); break;
    case 3: hipLaunchKernelGGL(k_dense_from_stencil<3>, dim3(g), dim3(kBlock), 0, st, S, J, K, A); break;
    case 4: hipLaunchKernelGGL(k_dense_from_stencil<4>, dim3(g), dim3(kBlock), 0, st, S, J, K, A); break;
    case 5: hipLaunchKernelGGL(k_dense_from_stencil<5>, dim3(g), dim3(kBlock), 0, st, S, J, K, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gj_step(double* A, int K, int k, double* row, double* col, double* piv, hipStream_t st) {
  hipLaunchKernelGGL(k_gj_save, dim3(blocks_for(K)), dim3(kBlock), 0, st, A, K, k, row, col, piv);
  hipLaunchKernelGGL(k_gj_update, dim3(blocks_for(int64_t(K) * K)), dim3(kBlock), 0, st, A, K, k, row, col);
  return hipGetLastError();
}
hipError_t launch_symmetrize(double* A, int K, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3(blocks_for(int64_t(K) * K)), dim3(kBlock), 0, st, A, K);
  return hipGetLastError();
}

template <typename TB, typename TV, typename TO>
hipError_t launch_gemv(const double* A, int K, const TB* base, double s, const TV* v, TO* out, hipStream_t st) {
  const unsigned g = unsigned((int64_t(K) * 64 + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_gemv<TB, TV, TO>), dim3(g), dim3(kBlock), 0, st, A, K, base, s, v, out);
  return hipGetLastError();
}
template hipError_t launch_gemv<double, double, double>(const double*, int, const double*, double, const double*,
                                                        double*, hipStream_t);
template hipError_t launch_gemv<double, float, double>(const double*, int, const double*, double, const float*,
                                                       double*, hipStream_t);
template hipError_t launch_gemv<float, double, double>(const double*, int, const float*, double, const double*,
                                                       double*, hipStream_t);
template hipError_t launch_gemv<double, double, float>(const double*, int, const double*, double, const double*,
                                                       float*, hipStream_t);

hipError_t launch_level_moments(int D, const double* t64, const uint32_t* cell, const int32_t* off, int64_t n,
                                int G, int g, double* mom, bool det, hipStream_t st) {
  int nrest = 1;
  for (int p = 1; p < D; ++p) nrest *= 7;
  const int nr = nrest < kBlock ? nrest : kBlock;
  const unsigned ncells = 1u << (D * g);
  const unsigned gy = ncells < 32768u ? ncells : 32768u;
  // split each cell's points so that the grid holds a few thousand blocks
  const unsigned gx = unsigned((nrest + nr - 1) / nr);
  int64_t chunks = (4096 + int64_t(gx) * gy - 1) / (int64_t(gx) * gy);
  const int64_t per_cell = n / int64_t(ncells) + 1;
  chunks = std::max<int64_t>(1, std::min<int64_t>({chunks, 1024, (per_cell + 255) / 256}));
  if (det) chunks = 1;   // one block per cell: no atomics, a fixed summation order
  const dim3 grid(gx, gy, unsigned(chunks));
  switch (D) {
    case 1: hipLaunchKernelGGL(k_level_moments<1>, grid, dim3(kBlock), 0, st, t64, cell, off, n, G, g, mom); break;
    case 2: hipLaunchKernelGGL(k_level_moments<2>, grid, dim3(kBlock), 0, st, t64, cell, off, n, G, g, mom); break;
    case 3: hipLaunchKernelGGL(k_level_moments<3>, grid, dim3(kBlock), 0, st, t64, cell, off, n, G, g, mom); break;
    case 4: hipLaunchKernelGGL(k_level_moments<4>, grid, dim3(kBlock), 0, st, t64, cell, off, n, G, g, mom); break;
    case 5: hipLaunchKernelGGL(k_level_moments<5>, grid, dim3(kBlock), 0, st, t64, cell, off, n, G, g, mom); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_moments_coarsen(const double* in, double* out, int Nc, int64_t outer, int64_t inner,
                                  hipStream_t st) {
  const int64_t total = outer * 7 * Nc * inner;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_moments_coarsen, dim3(blocks_for(total)), dim3(kBlock), 0, st, in, out, Nc, outer, inner);
  return hipGetLastError();
}

hipError_t launch_stencil_pass(const double* in, double* out, const double* ctab, int N, int64_t outer,
                               int64_t inner, hipStream_t st) {
  const int64_t total = outer * int64_t(7) * (N + kDeg) * inner;
  hipLaunchKernelGGL(k_stencil_pass, dim3(blocks_for(total)), dim3(kBlock), 0, st, in, out, ctab, N, inner, total);
  return hipGetLastError();
}

hipError_t launch_stencil_finalize(int D, const double* inter, const double* band, int J, int64_t K, double lam,
                                   double* S64, float* S32, hipStream_t st) {
  int64_t NO = 1;
  for (int p = 0; p < D; ++p) NO *= 7;
  const unsigned g = blocks_for((NO + 1) / 2 * K);   // the stored half
  switch (D) {
    case 1: hipLaunchKernelGGL(k_stencil_finalize<1>, dim3(g), dim3(kBlock), 0, st, inter, band, J, K, lam, S64, S32); break;
    case 2: hipLaunchKernelGGL(k_stencil_finalize<2>, dim3(g), dim3(kBlock), 0, st, inter, band, J, K, lam, S64, S32); break;
    case 3: hipLaunchKernelGGL(k_stencil_finalize<3>, dim3(g), dim3(kBlock), 0, st, inter, band, J, K, lam, S64, S32); break;
    case 4: hipLaunchKernelGGL(k_stencil_finalize<4>, dim3(g), dim3(kBlock), 0, st, inter, band, J, K, lam, S64, S32); break;
    case 5: hipLaunchKernelGGL(k_stencil_finalize<5>, dim3(g), dim3(kBlock), 0, st, inter, band, J, K, lam, S64, S32); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int EPI>
static hipError_t launch_stencil_epi(int D, const T* S, int J, const T* x, T* out, const T* b, const T* w,
                                     int64_t K, hipStream_t st) {
  if (K <= kStSmallMaxK) {
    const unsigned gs = unsigned((K + kStSmallRows - 1) / kStSmallRows);
    switch (D) {
      case 1: hipLaunchKernelGGL((k_stencil_apply_small<T, 1, EPI>), dim3(gs), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
      case 2: hipLaunchKernelGGL((k_stencil_apply_small<T, 2, EPI>), dim3(gs), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
      case 3: hipLaunchKernelGGL((k_stencil_apply_small<T, 3, EPI>), dim3(gs), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
      case 4: hipLaunchKernelGGL((k_stencil_apply_small<T, 4, EPI>), dim3(gs), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
      case 5: hipLaunchKernelGGL((k_stencil_apply_small<T, 5, EPI>), dim3(gs), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const unsigned g = unsigned((K + kStRows - 1) / kStRows);
  switch (D) {
    case 1: hipLaunchKernelGGL((k_stencil_apply<T, 1, EPI>), dim3(g), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
    case 2: hipLaunchKernelGGL((k_stencil_apply<T, 2, EPI>), dim3(g), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
    case 3: hipLaunchKernelGGL((k_stencil_apply<T, 3, EPI>), dim3(g), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
    case 4: hipLaunchKernelGGL((k_stencil_apply<T, 4, EPI>), dim3(g), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
    case 5: hipLaunchKernelGGL((k_stencil_apply<T, 5, EPI>), dim3(g), dim3(kBlock), 0, st, S, J, x, out, b, w, K); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil_apply(int D, int epi, const T* S, int J, const T* x, T* out, const T* b, const T* w,
                                int64_t K, hipStream_t st) {
  if (K == 0) return hipSuccess;
  if (epi == kStPlain) return launch_stencil_epi<T, kStPlain>(D, S, J, x, out, b, w, K, st);
  if (epi == kStJacobi) return launch_stencil_epi<T, kStJacobi>(D, S, J, x, out, b, w, K, st);
  if (epi == kStResidual) return launch_stencil_epi<T, kStResidual>(D, S, J, x, out, b, w, K, st);
  if (epi == kStJacobiZero) return launch_stencil_epi<T, kStJacobiZero>(D, S, J, x, out, b, w, K, st);
  return hipErrorInvalidValue;
}

template <typename T, int D>
static hipError_t launch_stencil_color_d(const T* S, int J, T* x, const T* b, T omega, int color, int64_t K,
                                         hipStream_t st) {
  int64_t rows = 1;
  int col = color;
  for (int p = D - 1; p >= 0; --p) {
    const int cp = col % 4;
    col /= 4;
    rows *= (J - cp + 3) / 4;
  }
  if (rows <= 0) return hipSuccess;
  const unsigned nb = unsigned((rows + kStSmallRows - 1) / kStSmallRows);
  hipLaunchKernelGGL((k_stencil_color<T, D>), dim3(nb), dim3(kBlock), 0, st, S, J, x, b, omega, color, rows, K);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil_color(int D, const T* S, int J, T* x, const T* b, T omega, int color, int64_t K,
                                hipStream_t st) {
  switch (D) {
    case 1: return launch_stencil_color_d<T, 1>(S, J, x, b, omega, color, K, st);
    case 2: return launch_stencil_color_d<T, 2>(S, J, x, b, omega, color, K, st);
    case 3: return launch_stencil_color_d<T, 3>(S, J, x, b, omega, color, K, st);
    case 4: return launch_stencil_color_d<T, 4>(S, J, x, b, omega, color, K, st);
    case 5: return launch_stencil_color_d<T, 5>(S, J, x, b, omega, color, K, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_stencil_color<double>(int, const double*, int, double*, const double*, double, int,
                                                 int64_t, hipStream_t);
template hipError_t launch_stencil_color<float>(int, const float*, int, float*, const float*, float, int, int64_t,
                                                hipStream_t);
template hipError_t launch_stencil_apply<double>(int, int, const double*, int, const double*, double*,
                                                 const double*, const double*, int64_t, hipStream_t);
template hipError_t launch_stencil_apply<float>(int, int, const float*, int, const float*, float*, const float*,
                                                const float*, int64_t, hipStream_t);

}  // namespace tsmg
