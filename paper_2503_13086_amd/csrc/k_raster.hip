// Tile rasterizer forward and backward for gfx950.
//
// Forward (Sec. III Eq. 2): one workgroup of T x T threads per T x T tile
// (T = 8, 16 or 32), one thread per pixel, each wavefront owning an 8x8 block.
// The tile's depth-ordered list is walked in batches of T^2 records staged in LDS;
// every pixel reads each staged record by LDS broadcast, so a record fetched from
// HBM once serves the whole tile.  Each wavefront tests the staged batch against
// its block (one record per lane, one ballot per 64 records: does the cutoff
// ellipse meet the block's pixel centres) and walks only the records that do.  A wavefront stops when all its pixels have stopped
// blending, the workgroup when all have.  Screen centres arrive in FP64 and are
// made relative to the tile origin while staging, so per-pixel offsets are
// accurate fp32 numbers at any image size.
//
// Backward (Sec. IV-E): the same tiling and per-block candidate sets, walking each
// list back to front from the last position any pixel of the tile blended (each
// wavefront starts at the last position its own pixels blended).  Each pixel
// recovers its transmittance with one reciprocal per Gaussian and keeps the colour
// accumulated behind it.  Per Gaussian, nine per-pixel values (the moments of
// dL/d(exponent) over dx, dy, dx^2, dx dy, dy^2, then opacity and colour partials)
// are summed across the wavefront by a reduce-scatter (CDNA4 permlane swaps across
// halves and row pairs, then DPP exchanges within rows; the Gaussians a wavefront
// blends are taken two at a time, sharing the last levels) and across the wavefronts
// with LDS adds; the moments become centre and conic partials once per tile, and each
// workgroup issues one global atomic per (tile, Gaussian, component) instead of
// one per (pixel, Gaussian, component), consecutive lanes taking consecutive
// components so a wavefront's atomics share cache lines.  Wavefronts in which no
// pixel blended a Gaussian skip it.
#include "gs_internal.h"

#pragma clang fp contract(off)

namespace gsk {
namespace {

// Wave-wide mask of a per-lane predicate (the compiler keeps the predicate in a
// scalar mask instead of round-tripping it through a vector register).
__device__ inline uint64_t wave_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }


// Tile of workgroup b.  Workgroups are dealt to the chip's 8 XCDs round-robin (b
// runs on XCD b mod 8, each XCD with its own L2); XCD x takes the runs x, x + 8,
// ... of 32 consecutive tiles, so neighbouring tiles, which stage mostly the same
// records, meet in one L2, while the short runs keep the work per XCD even (1%
// faster backward than plain tile order; whole contiguous eighths were slower).
// The grid is rounded up to whole rounds of runs; workgroups past the last tile
// return at once.
constexpr int kXcdRun = 32;
__device__ inline int xcd_raster_tile(int b) {
  const int x = b % 8, q = b / 8;
  return ((q / kXcdRun) * 8 + x) * kXcdRun + q % kXcdRun;
}

__device__ inline int view_of_tile(const ViewDev* __restrict__ views, int V, int tile) {
  int v = 0;
  while (v + 1 < V && tile >= views[v + 1].tile_off) ++v;
  return v;
}

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Base-2 exponent of the 2D Gaussian at offset (dx, dy): with A = -a/2, B = -b,
// C = -c/2 pre-scaled by log2(e), e^power = 2^result, taken as
// dx (A dx + B dy) + C dy^2 (five operations).
__device__ inline float gauss_power2(float A, float B, float C, float dx, float dy) {
  return __fmaf_rn(C * dy, dy, dx * __fmaf_rn(B, dy, A * dx));
}

struct TileGeom {
  int v, tx, ty, lx, ly, px, py;
  bool inside;
  double ox, oy;
};

template <int T>
__device__ inline TileGeom tile_geom(const ViewDev* __restrict__ views, int V, int tile) {
  TileGeom t;
  t.v = view_of_tile(views, V, tile);
  const ViewDev& cv = views[t.v];
  const int lt = tile - cv.tile_off;
  t.tx = lt % cv.tiles_x;
  t.ty = lt / cv.tiles_x;
  // wavefront w covers the 8x8 block (w mod T/8, w div T/8) of the tile; lane l
  // its pixel (l & 7, l >> 3)
  constexpr int QW = T / 8;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  t.lx = ((w % QW) << 3) | (l & 7);
  t.ly = ((w / QW) << 3) | (l >> 3);
  t.px = t.tx * T + t.lx;
  t.py = t.ty * T + t.ly;
  t.inside = t.px < cv.W && t.py < cv.H;
  t.ox = (double)(t.tx * T) + 0.5;
  t.oy = (double)(t.ty * T) + 0.5;
  return t;
}

// Stage record `rid` for a tile with origin (ox, oy): centre relative to the tile,
// exponent coefficients and cutoff in base-2 units (the exponent's sign and the
// cutoff test are unchanged by the positive factor), opacity, colour, and two
// values for the block test below: the slope kC = -b / c of the line on which the
// exponent peaks along vertical lines, and a cutoff tau_c = tau' (1 + 1e-5 kappa)
// slightly below the pixel test's, kappa = (sqrt(ac) + |b|)^2 / (ac - b^2) bounding
// (|A dx^2| + |B dx dy| + |C dy^2|) / |exponent|, so that fp32 rounding in either
// test can never make the block test drop a Gaussian a pixel accepts.  det = ac - b^2
// is one fused multiply-add (error below ulp(b^2), so below 2e-4 det wherever
// kappa < 1e4, and every conic with det <= 0 yields det < ulp(b^2), kappa > 1e4);
// kappa and kC are fp32 too (their errors only move the margin by as much of itself).
// A conic that is not clearly positive definite (det <= 0 or kappa >= 1e4) gets
// tau_c = -inf, so every block lists it.
//   q0 = (u', w', A, B)   q1 = (C, tau', tau_c, kC)   q2 = (o, r, g, b)
// (the per-pixel test reads q0 and q1.xy, a blend q2).
__device__ inline void stage(const Record* __restrict__ rec, uint32_t rid, double ox, double oy, float4& q0,
                             float4& q1, float4& q2) {
  const Record* r = rec + rid;
  const double2 uw = *reinterpret_cast<const double2*>(r);
  const float4 c = reinterpret_cast<const float4*>(r)[1];
  const float4 d = reinterpret_cast<const float4*>(r)[2];
  const float det = __fmaf_rn(c.x, c.z, -(c.y * c.y));
  const float tau2 = d.x * kLog2e;
  float tc = -INFINITY, kc = 0.0f;
  if (det > 0.0f) {
    const float s = __builtin_amdgcn_sqrtf(c.x * c.z) + fabsf(c.y);
    const float kappa = (s * s) * __builtin_amdgcn_rcpf(det);
    if (kappa < 1e4f) tc = tau2 * (1.0f + 1e-5f * kappa);
    kc = -c.y * __builtin_amdgcn_rcpf(c.z);
  }
  q0 = make_float4((float)(uw.x - ox), (float)(uw.y - oy), (-0.5f * c.x) * kLog2e, (-c.y) * kLog2e);
  q1 = make_float4((-0.5f * c.z) * kLog2e, tau2, tc, kc);
  q2 = make_float4(c.w, d.y, d.z, d.w);
}

// Placeholder for an entry that belongs to no Gaussian (never for a consistent
// sort): no pixel accepts it and no block lists it.
__device__ inline void stage_empty(float4& q0, float4& q1, float4& q2) {
  q0 = make_float4(0.f, 0.f, 0.f, 0.f);
  q1 = make_float4(0.f, 1.f, INFINITY, 0.f);
  q2 = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Ballots of the staged records [0, m) whose cutoff ellipse meets this wavefront's
// 8x8 block of pixel centres [qx, qx + 7] x [qy, qy + 7] (tile-relative); bit b
// of mask[k] is record 64 k + b.  The pixels' offsets u' - x, w' - y fill the box
// [x0, x1] x [y0, y1] (same fp32 subtractions as the pixel test), and the largest
// exponent over that box lies on the edge dx = xn (the box's nearest value to 0),
// where it peaks at dy = kC xn, or on the edge dy = yn, peak dx = kA yn (a concave
// quadratic's maximum over a box is at its centre, or on an edge next to the
// nearest corner); any point of the box bounds that maximum from below, so the
// rounding of the peak positions only costs the second-order loss already
// covered by tau_c.
template <int NM>
__device__ inline void block_masks(const float4* s0, const float4* s1, int m, float qx, float qy,
                                      uint64_t (&mask)[NM]) {
  const int lane = (int)__lane_id();
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    const int j = lane + 64 * k;
    bool hit = false;
    if (j < m) {
      const float4 a0 = s0[j];
      const float4 a1 = s1[j];
      const float x0 = a0.x - (qx + 7.0f), x1 = a0.x - qx;
      const float y0 = a0.y - (qy + 7.0f), y1 = a0.y - qy;
      // (x0 <= x1 and y0 <= y1: a median of three is a clamp)
      const float xn = __builtin_amdgcn_fmed3f(0.0f, x0, x1);
      const float yn = __builtin_amdgcn_fmed3f(0.0f, y0, y1);
      const float ka = (-0.5f * a0.w) * __builtin_amdgcn_rcpf(a0.z);
      const float dy1 = __builtin_amdgcn_fmed3f(xn * a1.w, y0, y1);
      const float dx2 = __builtin_amdgcn_fmed3f(yn * ka, x0, x1);
      const float f1 = gauss_power2(a0.z, a0.w, a1.x, xn, dy1);
      const float f2 = gauss_power2(a0.z, a0.w, a1.x, dx2, yn);
      hit = fmaxf(f1, f2) >= a1.z;
    }
    mask[k] = wave_mask(hit);
  }
}

// COUNT: the same walk, writing only the number of Gaussians each pixel evaluated up
// to its termination (those that pass its cutoff test: the blended ones and, if it
// stopped, the one that stopped it) into evals, and the number of the tile's list
// entries that at least one of its pixels blended into pairs_eff[tile]; the forward
// state is left alone.
template <int T, bool COUNT = false>
__global__ __launch_bounds__(T * T) void k_render_fwd(const ViewDev* __restrict__ views, int V, int n_tiles_total,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ pair_rec,
                                                    const Record* __restrict__ rec, uint32_t n_rec,
                                                    float* __restrict__ color,
                                                    float* __restrict__ t_final, uint32_t* __restrict__ n_contrib,
                                                    uint32_t* __restrict__ last, float* __restrict__ asum,
                                                    uint32_t* __restrict__ evals = nullptr,
                                                    uint32_t* __restrict__ pairs_eff = nullptr) {
  constexpr int NT = T * T, NM = NT / 64;
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  __shared__ uint32_t s_eff[COUNT ? NT / 32 : 1];   // batch entries some pixel blended (COUNT)
  uint32_t n_eff = 0;
  const int tile = xcd_raster_tile((int)blockIdx.x);
  if (tile >= n_tiles_total) return;
  const TileGeom tg = tile_geom<T>(views, V, tile);
  const uint2 rg = ranges[tile];
  const float fx = (float)tg.lx, fy = (float)tg.ly;
  const float qx = (float)(tg.lx & ~7), qy = (float)(tg.ly & ~7);
  float Tr = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, A = 0.0f;
  uint32_t cnt = 0, lastp = 0;
  // A pixel takes a Gaussian while its exponent lies in [cutoff, pmax]: pmax is 0
  // while the pixel blends and -inf once it has stopped (or lies outside the
  // image), which keeps the test two plain comparisons.
  float pmax = tg.inside ? 0.0f : -INFINITY;
  for (uint32_t base = rg.x; base < rg.y; base += NT) {
    const uint32_t m = min((uint32_t)NT, rg.y - base);
    __syncthreads();
    if (COUNT && threadIdx.x < NT / 32) s_eff[threadIdx.x] = 0u;
    if (threadIdx.x < m) {
      const uint32_t rid = pair_rec[base + threadIdx.x];
      if (rid < n_rec) {
        stage(rec, rid, tg.ox, tg.oy, s0[threadIdx.x], s1[threadIdx.x], s2[threadIdx.x]);
      } else {
        stage_empty(s0[threadIdx.x], s1[threadIdx.x], s2[threadIdx.x]);
      }
    }
    __syncthreads();
    if (wave_mask(pmax == 0.0f) != 0ull) {
      uint64_t mask[NM];
      block_masks<NM>(s0, s1, (int)m, qx, qy, mask);
      // straight-line per-Gaussian update; lanes that skip or have stopped keep their state
      const uint32_t pos0 = base - rg.x + 1;
      bool live = true;
      for (int k = 0; k < NM && live; ++k) {
        uint64_t mk = mask[k];
        while (mk) {
          const uint32_t j = 64u * k + (uint32_t)__builtin_ctzll(mk);
          mk &= mk - 1ull;
          const float4 a0 = s0[j];
          const float4 a1 = s1[j];
          const float dx = a0.x - fx, dy = a0.y - fy;
          const float p2 = gauss_power2(a0.z, a0.w, a1.x, dx, dy);
          const bool pass = p2 <= pmax && p2 >= a1.y;
          if (wave_mask(pass) != 0ull) {
            const float4 a2 = s2[j];
            const float alpha = fminf(kAlphaMax, a2.x * __builtin_amdgcn_exp2f(p2));
            const float Tn = Tr * (1.0f - alpha);
            const bool stop = pass && Tn < kTMin;
            const bool blend = pass && !stop;
            pmax = stop ? -INFINITY : pmax;
            const float ab = blend ? alpha : 0.0f;  // this pixel's alpha, 0 if it did not blend
            const float wgt = ab * Tr;
            C0 = __fmaf_rn(a2.y, wgt, C0);
            C1 = __fmaf_rn(a2.z, wgt, C1);
            C2 = __fmaf_rn(a2.w, wgt, C2);
            Tr = blend ? Tn : Tr;
            A += ab;
            cnt += blend ? 1u : 0u;
            lastp = blend ? pos0 + j : lastp;
            if (COUNT && wave_mask(blend) != 0ull && __lane_id() == 0u) atomicOr(&s_eff[j >> 5], 1u << (j & 31u));
            // leave the batch once every pixel of this wavefront has stopped
            mk = wave_mask(pmax == 0.0f) == 0ull ? 0ull : mk;
          }
        }
        live = wave_mask(pmax == 0.0f) != 0ull;
      }
    }
    if (COUNT) {
      __syncthreads();
      if (threadIdx.x == 0)
        for (int w = 0; w < NT / 32; ++w) n_eff += (uint32_t)__popc(s_eff[w]);
    }
    if (__syncthreads_and(pmax < 0.0f)) break;
  }
  if (COUNT) {
    if (tg.inside) {
      const ViewDev& cv = views[tg.v];
      evals[(size_t)cv.pix_off + (size_t)tg.py * cv.W + tg.px] = cnt + (pmax < 0.0f ? 1u : 0u);
    }
    if (threadIdx.x == 0) pairs_eff[tile] = n_eff;
    return;
  }
  if (tg.inside) {
    const ViewDev& cv = views[tg.v];
    const size_t hw = (size_t)cv.W * cv.H;
    const size_t pix = (size_t)tg.py * cv.W + tg.px;
    float* img = color + 3 * (size_t)cv.pix_off;
    img[pix] = C0 + Tr * cv.bg[0];
    img[hw + pix] = C1 + Tr * cv.bg[1];
    img[2 * hw + pix] = C2 + Tr * cv.bg[2];
    const size_t gp = (size_t)cv.pix_off + pix;
    t_final[gp] = Tr;
    n_contrib[gp] = cnt;
    last[gp] = lastp;
    asum[gp] = A;
  }
}

// a + b across the two halves of the wave: lanes 0-31 receive the sum of a over
// lanes l and l + 32, lanes 32-63 the sum of b (v_permlane32_swap, CDNA4).
__device__ inline float fold32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The same across row pairs: rows (0, 1) and (2, 3) of 16 lanes; row 0 and row 2
// keep a, rows 1 and 3 keep b (v_permlane16_swap, CDNA4).
__device__ inline float fold16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// x plus lane l ^ 16's x (the partner row within each half of the wave), through the
// LDS crossbar (ds_swizzle, no memory access) rather than a VALU swap: the ninth
// values need only the rows that the even rows end up with.
__device__ inline float add_row_pair(float x) {
  // bit mode: and_mask 0x1f, or_mask 0, xor_mask 0x10
  return x + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x401F));
}

// Lane l receives v from the lane the DPP control names (row_ror:8 = 0x128: lane
// l ^ 8 of its row; row_half_mirror = 0x141: lane 7 - l of its half-row;
// quad_perm [2,3,0,1] = 0x4E and [1,0,3,2] = 0xB1: lanes l ^ 2 and l ^ 1).
template <int CTRL>
__device__ inline float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

// a + b across the partner lanes of a DPP permutation that pairs each lane with
// one whose selector bit `hi` differs: lanes with hi clear keep the sum of a over
// the pair, lanes with hi set the sum of b.
template <int CTRL>
__device__ inline float fold_dpp(float a, float b, bool hi) {
  const float own = hi ? b : a, give = hi ? a : b;
  return own + dpp<CTRL>(give);
}

// fold_dpp for a selector that is a DPP bank bit (bit 3: banks 2 and 3 of each row;
// bit 2: banks 1 and 3), without the two selects: every lane forms a plus its
// partner's a, then the lanes of the selected banks overwrite that with b plus the
// partner's b (a DPP add that writes those banks only).  A DPP read of a VGPR that
// the VALU wrote in the last two cycles needs two wait states, and the compiler
// does not see inside the asm: the nops before and after cover the asm's own read
// and any DPP read of its result.  The same sums in the same order as fold_dpp.
__device__ inline float fold_ror8_bit3(float a, float b) {
  float t = a + dpp<0x128>(a);
  asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 row_ror:8 row_mask:0xf bank_mask:0xc bound_ctrl:1\n\ts_nop 1" : "+v"(t) : "v"(b));
  return t;
}
__device__ inline float fold_mirror_bit2(float a, float b) {
  float t = a + dpp<0x141>(a);
  asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xa bound_ctrl:1\n\ts_nop 1" : "+v"(t) : "v"(b));
  return t;
}

// Reduce-scatter of nine per-lane values over the wave, added into an LDS row.
// Each level halves the registers by pairing lanes whose selector bit differs
// (across wave halves, across row pairs, across half-rows, across the halves of
// each half-row by mirroring), then quad permutations finish the sums.  The first
// eight values go through the first three levels on their own (reduce8_part);
// the ninth joins there.  A record alone (reduce9_tail) ends with every group of
// four lanes holding one total, and the lane of each group with slot >= 0 adds it
// into LDS (nine lanes, one instruction): with r = row, h = lane bit 3, q = lane
// bit 2, value {0, 2, 1, 3}[r] + 4h sits where q = 0 and value 8 where r = h = 0,
// q = 1.  Two records (reduce18_tail) share the last three levels: every pair of
// lanes then holds one of the 18 totals (the second record's at lane bit 2 set,
// both ninth values at lane bit 1 set), which costs 45 instructions instead of 56.
typedef __attribute__((address_space(3))) float LdsFloat;

__device__ inline float reduce8_part(const float (&v)[kGrad2D]) {
  const float b0 = fold32(v[0], v[1]);
  const float b1 = fold32(v[2], v[3]);
  const float b2 = fold32(v[4], v[5]);
  const float b3 = fold32(v[6], v[7]);
  const float c0 = fold16(b0, b1);
  const float c1 = fold16(b2, b3);
  return fold_ror8_bit3(c0, c1);
}

__device__ inline void lds_add(uint32_t addr, float x) {
  __hip_atomic_fetch_add((LdsFloat*)(uintptr_t)addr, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// d = reduce8_part of the record's first eight values, v8 its ninth; lanes with
// `add` add their total at addr (row and column included).
__device__ inline void reduce9_tail(float d, float v8, uint32_t addr, bool add) {
  const float c2 = add_row_pair(fold32(v8, 0.0f));
  const float d1 = c2 + dpp<0x128>(c2);
  float e = fold_mirror_bit2(d, d1);
  e += dpp<0x4E>(e);
  e += dpp<0xB1>(e);
  if (add) lds_add(addr, e);
}

// Records a and b (parts da, db, ninth values a8, b8) reduced together; lanes that
// hold a total of a add it at addr_a, those holding one of b at addr_b.
__device__ inline void reduce18_tail(float da, float a8, float db, float b8, uint32_t addr_a, uint32_t addr_b,
                                     bool add_a, bool add_b, bool bit1) {
  const float m2 = add_row_pair(fold32(a8, b8));
  const float m3 = m2 + dpp<0x128>(m2);
  const float e0 = fold_mirror_bit2(da, db);
  const float e1 = m3 + dpp<0x141>(m3);
  float f = fold_dpp<0x4E>(e0, e1, bit1);
  f += dpp<0xB1>(f);
  if (add_a) lds_add(addr_a, f);
  if (add_b) lds_add(addr_b, f);
}

// Byte offset of row j of the [NT][kGrad2D] float accumulator, formed on the scalar
// unit (j is uniform); left to itself the compiler folds it into a 64-bit vector
// multiply-add of the lane's address.
__device__ inline uint32_t acc_row_offset(int j) {
  static_assert(kGrad2D * sizeof(float) == 36, "accumulator row size");
  uint32_t off;
  asm("s_mul_i32 %0, %1, 36" : "=s"(off) : "s"(__builtin_amdgcn_readfirstlane(j)));
  return off;
}

// The accumulator column reduce9_tail adds from this lane (-1: none).
__device__ inline int reduce9_slot(unsigned lane) {
  if (lane & 3u) return -1;
  const unsigned r = lane >> 4, h = (lane >> 3) & 1u, q = (lane >> 2) & 1u;
  if (q == 0u) return (int)((((r & 1u) << 1) | (r >> 1)) + 4u * h);
  return (r == 0u && h == 0u) ? 8 : -1;
}

// The total reduce18_tail leaves in this lane for it to add: 0-8 for the first
// record's columns, 9-17 for the second's (-1: none).
__device__ inline int reduce18_slot(unsigned lane) {
  if (lane & 1u) return -1;
  const unsigned r = lane >> 4, h = (lane >> 3) & 1u, q = (lane >> 2) & 1u;
  if ((lane & 2u) == 0u) return (int)((((r & 1u) << 1) | (r >> 1)) + 4u * h + 9u * q);
  if (h == 0u && q == 0u && (r & 1u) == 0u) return r == 0u ? 8 : 17;
  return -1;
}

// ORDERED: instead of adding each (tile, Gaussian) partial sum into grad2d with a
// global atomic, write it to out[pair position * kGrad2D + component] (every
// position of the tile's list, zeros included), each wave reducing into its own
// LDS rows and the waves' rows summed in wave order, so that every partial is the
// same bits on every run; the per-Gaussian sums are then taken in tile order by
// launch_ordered_sum.
template <int T, bool ORDERED = false>
__global__ __launch_bounds__(T * T) void k_render_bwd(const ViewDev* __restrict__ views, int V, int n_tiles_total,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ pair_rec,
                                                    const Record* __restrict__ rec, uint32_t n_rec,
                                                    const float* __restrict__ t_final,
                                                    const uint32_t* __restrict__ last,
                                                    const float* __restrict__ dL_dcolor,
                                                    const float* __restrict__ dL_dG, float* __restrict__ grad2d) {
  // records are staged NB at a time, half the tile's threads (at least 64): 11 KB of
  // LDS at T = 16, so registers rather than LDS set the occupancy (8 waves per SIMD)
  // (the ordered mode keeps one accumulator per wave: 64 records per batch)
  constexpr int NT = T * T, NB = ORDERED ? 64 : (NT >= 128 ? NT / 2 : NT), NM = NB / 64, NW = NT / 64;
  __shared__ float4 s0[NB], s1[NB], s2[NB];
  __shared__ uint32_t srid[NB];
  constexpr int NACC = ORDERED ? NW : 1;
  __shared__ float acc[NACC][NB][kGrad2D];
  __shared__ uint32_t smax[NW];
  const int tile = xcd_raster_tile((int)blockIdx.x);
  if (tile >= n_tiles_total) return;
  const TileGeom tg = tile_geom<T>(views, V, tile);
  const ViewDev& cv = views[tg.v];
  const uint2 rg = ranges[tile];
  const float fx = (float)tg.lx, fy = (float)tg.ly;
  const float qx = (float)(tg.lx & ~7), qy = (float)(tg.ly & ~7);

  // Sg = sum over channels of dL/dcolour times the colour accumulated behind the
  // current Gaussian (background included): the only form in which that colour
  // enters dL/dalpha.
  float Tr = 0.0f, Sg = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gG = 0.0f;
  uint32_t lp = 0;
  if (tg.inside) {
    const size_t hw = (size_t)cv.W * cv.H;
    const size_t pix = (size_t)tg.py * cv.W + tg.px;
    const size_t gp = (size_t)cv.pix_off + pix;
    Tr = t_final[gp];
    lp = last[gp];
    const float* gimg = dL_dcolor + 3 * (size_t)cv.pix_off;
    g0 = gimg[pix];
    g1 = gimg[hw + pix];
    g2 = gimg[2 * hw + pix];
    if (dL_dG) gG = dL_dG[gp];
    Sg = Tr * __fmaf_rn(g2, cv.bg[2], __fmaf_rn(g1, cv.bg[1], g0 * cv.bg[0]));
  }
  uint32_t mx = lp;
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
  const int wave_last = (int)mx;           // this wave never needs list positions >= wave_last
  const unsigned lane = __lane_id();
  const int slot = reduce9_slot(lane), slot18 = reduce18_slot(lane);
  const bool bit1 = (lane & 2u) != 0u;
  const bool add9 = slot >= 0, add_a = slot18 >= 0 && slot18 < kGrad2D, add_b = slot18 >= kGrad2D;
  // 32-bit LDS byte addresses of this lane's columns in acc[0] for the two
  // reductions (plain integer arithmetic in the loop: the compiler would otherwise
  // form the address in 64 bits)
  const uint32_t acc0 = (uint32_t)(uintptr_t)(LdsFloat*)&acc[ORDERED ? threadIdx.x / 64 : 0][0][0];
  const uint32_t col9 = acc0 + 4u * (uint32_t)(slot < 0 ? 0 : slot);
  const uint32_t col18 = acc0 + 4u * (uint32_t)(slot18 < 0 ? 0 : slot18 % kGrad2D);
  if (__lane_id() == 0) smax[threadIdx.x / 64] = mx;
  for (int i = threadIdx.x; i < NACC * NB * kGrad2D; i += NT) (&acc[0][0][0])[i] = 0.0f;
  __syncthreads();
  int jmax = 0;
  for (int w = 0; w < NW; ++w) jmax = max(jmax, (int)smax[w]);

  for (int end = jmax; end > 0; end -= NB) {
    const int beg = end > NB ? end - NB : 0;
    const int m = end - beg;
    __syncthreads();
    if ((int)threadIdx.x < m) {
      const uint32_t rid = pair_rec[rg.x + beg + threadIdx.x];
      srid[threadIdx.x] = rid;
      if (rid < n_rec) {
        stage(rec, rid, tg.ox, tg.oy, s0[threadIdx.x], s1[threadIdx.x], s2[threadIdx.x]);
      } else {
        stage_empty(s0[threadIdx.x], s1[threadIdx.x], s2[threadIdx.x]);
      }
    }
    __syncthreads();
    // records this wavefront may need: positions below its own last blended one
    // whose cutoff ellipse meets its block, walked back to front
    uint64_t mask[NM];
    block_masks<NM>(s0, s1, min(m, wave_last - beg), qx, qy, mask);
    const uint32_t lrel = lp > (uint32_t)beg ? lp - (uint32_t)beg : 0u;   // batch positions this pixel blended
    for (int k = NM - 1; k >= 0; --k) {
      uint64_t mk = mask[k];
      // blended records are reduced two at a time: the first waits (as the first
      // three levels of its reduction and its ninth value) for the next
      float da = 0.0f, a8 = 0.0f;
      int ja = -1;
      while (mk) {
        const int b = 63 - __builtin_clzll(mk);
        mk &= ~(1ull << b);
        const int j = 64 * k + b;
        const float4 a0 = s0[j];
        const float4 a1 = s1[j];
        const float4 a2 = s2[j];
        const float dx = a0.x - fx, dy = a0.y - fy;
        const float p2 = gauss_power2(a0.z, a0.w, a1.x, dx, dy);
        const bool on = (uint32_t)j < lrel && p2 <= 0.0f && p2 >= a1.y;
        // (a2 is fetched with a0 and a1, before the branch: one address, and the blend
        // below waits for nothing more)
        asm volatile("" ::"v"(a2.x), "v"(a2.y), "v"(a2.z), "v"(a2.w));
        if (wave_mask(on) == 0ull) continue;    // no pixel of this wave blended it
        // straight-line update; lanes that did not blend this Gaussian keep their state
        // and contribute zeros
        const float G = __builtin_amdgcn_exp2f(p2);
        const float og = a2.x * G;
        const bool capped = og > kAlphaMax;
        // alpha of this pixel, 0 where it did not blend: then 1 / (1 - alpha) = 1
        // exactly and transmittance and weight need no select
        const float alpha = on ? fminf(og, kAlphaMax) : 0.0f;
        const float ri = __builtin_amdgcn_rcpf(1.0f - alpha);
        Tr = Tr * ri;                          // transmittance in front of this Gaussian
        const float wgt = alpha * Tr;
        // Per pixel: colour partials, opacity partial and the moments of the exponent's
        // derivative dpow over (dx, dy, dx^2, dx dy, dy^2); the centre and conic
        // partials are fixed linear maps of these moments (applied once per tile).
        // dL/dalpha = T (g . colour) - Sg / (1 - alpha) + gG, gG being the
        // load-balancing gradient of the pixel's soft count (each blended alpha enters
        // it with weight 1).
        const float cg = __fmaf_rn(g2, a2.w, __fmaf_rn(g1, a2.z, g0 * a2.y));
        float dLda = __fmaf_rn(Tr, cg, __fmaf_rn(-Sg, ri, gG));
        dLda = (on && !capped) ? dLda : 0.0f;  // a capped alpha has zero derivative
        Sg = __fmaf_rn(cg, wgt, Sg);
        const float dpow = dLda * og;           // dL/d(exponent)
        float p[kGrad2D];
        p[0] = dpow * dx;
        p[1] = dpow * dy;
        p[2] = p[0] * dx;
        p[3] = p[0] * dy;
        p[4] = p[1] * dy;
        p[5] = dpow;                            // dL/dopacity = (sum of dpow) / o, formed per tile
        p[6] = g0 * wgt;
        p[7] = g1 * wgt;
        p[8] = g2 * wgt;
        const float d = reduce8_part(p);
        if (ja < 0) {
          da = d;
          a8 = p[8];
          ja = j;
        } else {
          reduce18_tail(da, a8, d, p[8], col18 + acc_row_offset(ja), col18 + acc_row_offset(j), add_a, add_b, bit1);
          ja = -1;
        }
      }
      if (ja >= 0) reduce9_tail(da, a8, col9 + acc_row_offset(ja), add9);
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      float* a = acc[0][threadIdx.x];
      if (ORDERED) {
        for (int w = 1; w < NACC; ++w)
          for (int k = 0; k < kGrad2D; ++k) a[k] += acc[w][threadIdx.x][k];
      }
      // moments -> partials: with exponent p = -(a dx^2 + 2 b dx dy + c dy^2)/2 and the
      // staged coefficients A, B, C = (-a/2, -b, -c/2) log2(e):
      // dp/du = ln2 (2A dx + B dy), dp/dw = ln2 (B dx + 2C dy),
      // dp/da = -dx^2/2, dp/db = -dx dy, dp/dc = -dy^2/2
      const float A = s0[threadIdx.x].z, B = s0[threadIdx.x].w, C = s1[threadIdx.x].x;
      const float m1 = a[0], m2 = a[1], m3 = a[2], m4 = a[3], m5 = a[4];
      a[0] = kLn2 * (2.0f * A * m1 + B * m2);
      a[1] = kLn2 * (B * m1 + 2.0f * C * m2);
      a[2] = -0.5f * m3;
      a[3] = -m4;
      a[4] = -0.5f * m5;
      // dL/dopacity: the exponent derivative summed over the tile's pixels is
      // sum dL/dalpha o G, so dividing by o gives sum dL/dalpha G
      const float o = s2[threadIdx.x].x;
      a[5] = o > 0.0f ? a[5] / o : 0.0f;
    }
    __syncthreads();
    // one global atomic per (tile, Gaussian, component); consecutive lanes take
    // consecutive components, so a wavefront's atomics fall on a few cache lines
    // (element offsets in 64 bits: n_rec * 9 may pass 2^32 bytes)
    float* af = &acc[0][0][0];
    if (ORDERED) {
      float* po = grad2d + ((size_t)rg.x + (size_t)beg) * kGrad2D;
      for (int i = threadIdx.x; i < m * kGrad2D; i += NT) po[i] = srid[i / kGrad2D] < n_rec ? af[i] : 0.0f;
      __syncthreads();
      for (int i = threadIdx.x; i < NACC * NB * kGrad2D; i += NT) af[i] = 0.0f;
    } else {
      for (int i = threadIdx.x; i < m * kGrad2D; i += NT) {
        const int j = i / kGrad2D;
        const uint32_t rid = srid[j];
        const float x = af[i];
        if (x != 0.0f && rid < n_rec)
          unsafeAtomicAdd(grad2d + ((size_t)rid * kGrad2D + (size_t)(i - kGrad2D * j)), x);
        af[i] = 0.0f;
      }
    }
  }
  if (ORDERED) {
    // list positions no pixel of the tile reached: zero partials
    const size_t len = rg.y > rg.x ? (size_t)(rg.y - rg.x) : 0;
    float* po = grad2d + (size_t)rg.x * kGrad2D;
    for (size_t i = (size_t)jmax * kGrad2D + threadIdx.x; i < len * kGrad2D; i += NT) po[i] = 0.0f;
  }
}

}  // namespace

hipError_t launch_render_fwd(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                             const Record* rec, uint32_t n_rec, float* color, float* t_final, uint32_t* n_contrib,
                             uint32_t* last, float* asum, int tile, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n_tiles + 8 * kXcdRun - 1) / (8 * kXcdRun) * (8 * kXcdRun)));
  switch (tile) {
    case 8:
      hipLaunchKernelGGL(k_render_fwd<8>, grid, dim3(64), 0, s, views, V, n_tiles, ranges, pair_rec, rec, n_rec, color, t_final,
                         n_contrib, last, asum);
      break;
    case 16:
      hipLaunchKernelGGL(k_render_fwd<16>, grid, dim3(256), 0, s, views, V, n_tiles, ranges, pair_rec, rec, n_rec, color,
                         t_final, n_contrib, last, asum);
      break;
    case 32:
      hipLaunchKernelGGL(k_render_fwd<32>, grid, dim3(1024), 0, s, views, V, n_tiles, ranges, pair_rec, rec, n_rec, color,
                         t_final, n_contrib, last, asum);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_render_count(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                               const Record* rec, uint32_t n_rec, uint32_t* evals, uint32_t* pairs_eff, int tile,
                               hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n_tiles + 8 * kXcdRun - 1) / (8 * kXcdRun) * (8 * kXcdRun)));
  switch (tile) {
    case 8:
      hipLaunchKernelGGL((k_render_fwd<8, true>), grid, dim3(64), 0, s, views, V, n_tiles, ranges, pair_rec, rec, n_rec,
                         nullptr, nullptr, nullptr, nullptr, nullptr, evals, pairs_eff);
      break;
    case 16:
      hipLaunchKernelGGL((k_render_fwd<16, true>), grid, dim3(256), 0, s, views, V, n_tiles, ranges, pair_rec, rec,
                         n_rec, nullptr, nullptr, nullptr, nullptr, nullptr, evals, pairs_eff);
      break;
    case 32:
      hipLaunchKernelGGL((k_render_fwd<32, true>), grid, dim3(1024), 0, s, views, V, n_tiles, ranges, pair_rec, rec,
                         n_rec, nullptr, nullptr, nullptr, nullptr, nullptr, evals, pairs_eff);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_render_bwd(const ViewDev* views, int V, int n_tiles, const uint2* ranges, const uint32_t* pair_rec,
                             const Record* rec, uint32_t n_rec, const float* t_final, const uint32_t* last,
                             const float* dL_dcolor, const float* dL_dG, float* grad2d, int tile, int ordered,
                             hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n_tiles + 8 * kXcdRun - 1) / (8 * kXcdRun) * (8 * kXcdRun)));
#define GS_BWD(TT, OO)                                                                                            \
  hipLaunchKernelGGL((k_render_bwd<TT, OO>), grid, dim3(TT * TT), 0, s, views, V, n_tiles, ranges, pair_rec, rec, \
                     n_rec, t_final, last, dL_dcolor, dL_dG, grad2d)
  switch (tile) {
    case 8: if (ordered) GS_BWD(8, true); else GS_BWD(8, false); break;
    case 16: if (ordered) GS_BWD(16, true); else GS_BWD(16, false); break;
    case 32: if (ordered) GS_BWD(32, true); else GS_BWD(32, false); break;
    default: return hipErrorInvalidValue;
  }
#undef GS_BWD
  return hipGetLastError();
}

}  // namespace gsk
