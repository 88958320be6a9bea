// Typed middle counts of the dense groups of the 4-cycle pass, bucketed by
// far-end id range and summed in LDS (Algorithm 2's 4-cycle orbit g6, from
// degree-ordered wedges).
//
// For a heavy node x, every cycle x-u-w-u' with x above u, u' and w in the
// degree order is found through its wedges x-u-w and x-u'-w; what a wedge
// needs is c_t(x, w), the number of middles of type t between x and w, kept
// in a dense row per far end w.  Instead of one global atomic per wedge into
// that row, the counts come from two kernels:
//   k_c4_bwalk: a walk item (at most CHW consecutive wedges of one node)
//     walks its wedges like the grouped kernel does (64 slots per window,
//     wedges dealt to lanes through a wavefront prefix sum) and writes each
//     wedge whose far end precedes x as a 4-byte record (offset of w inside
//     its id range of R ids, type of the middle), grouped by range, into the
//     item's own CHW words; runs[item][k] is where range k starts;
//   k_c4_bcount: one workgroup per (node, range) adds the range's records of
//     every item of the node into an LDS table of R rows (L 16-bit counts,
//     two per word) and writes out the rows of the far ends the node reaches
//     (4 words each); the credit walk reads no other row, so the array needs
//     no clearing.
// The credit walk of the grouped kernel then reads the rows as before.
//
// Needs L <= 8, 16-bit middle counts (every node of the group of degree below
// 65536: rows of 4 words, also where other groups keep 32-bit counts), the
// packed degree and type of every slot's column node (cdt), degrees below
// 2^28, CHW <= 32768 and at most CHW / 2 ranges.

namespace tg {

// LDS bytes of k_c4_bwalk: staged records and keys, the range histogram and
// a record counter.
__host__ __device__ inline size_t c4_bwalk_lds(int CHW, int K) {
  return (size_t)(2 * CHW + K + 4) * sizeof(uint32_t);
}

// Walk item b of a group belongs to the node gi with nit[gi] <= b <
// nit[gi + 1] (nit: the group's per-node item starts, Gg + 1 entries) and
// covers the node's wedges [CHW (b - nit[gi]), CHW (b - nit[gi] + 1)),
// clipped to the node's wedge count.
template <int NW>
__global__ void __launch_bounds__(NW * TG_WAVE) k_c4_bwalk(const int32_t* __restrict__ nit, int Gg, int CHW, int R,
                                                         int K, const int32_t* __restrict__ gx,
                                                         const int64_t* __restrict__ gslot,
                                                         const int64_t* __restrict__ wp,
                                                         const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const uint32_t* __restrict__ cdt,
                                                         uint32_t* __restrict__ region, int32_t* __restrict__ runs) {
  extern __shared__ uint32_t bw_lds[];
  uint32_t* srec = bw_lds;            // CHW staged records
  uint32_t* skey = bw_lds + CHW;      // CHW keys: range << 16 | rank inside the range
  uint32_t* hist = bw_lds + 2 * CHW;  // K
  uint32_t* nst = hist + K;
  const int wv = threadIdx.x / TG_WAVE, ln = lane();
  int gi = 0;
  {
    int a = 0, b = Gg;  // the largest gi with nit[gi] <= blockIdx.x
    while (b - a > 1) {
      const int mid = (a + b) >> 1;
      if (nit[mid] <= (int32_t)blockIdx.x) a = mid; else b = mid;
    }
    gi = a;
  }
  const int64_t sbase = gslot[0];
  const int64_t s_lo = gslot[gi] - sbase, s_hi = gslot[gi + 1] - sbase;  // the node's slots
  const int64_t W0 = wp[0];
  const int64_t item_wa = wp[s_lo] - W0 + (int64_t)((int32_t)blockIdx.x - nit[gi]) * CHW;
  const int64_t item_wb = min(wp[s_hi] - W0, item_wa + (int64_t)CHW);
  const int32_t x = gx[gi];
  const int32_t bx = rp[x], dx = rp[x + 1] - bx;
  for (int i = threadIdx.x; i < K; i += blockDim.x) hist[i] = 0u;
  if (threadIdx.x == 0) *nst = 0u;
  __syncthreads();
  // wavefront wv walks an equal share of the item's wedges
  const int64_t sub = (item_wb - item_wa + NW - 1) / NW;
  const int64_t wbeg = item_wa + wv * sub;
  const int64_t wend = min(item_wb, wbeg + sub);
  if (wbeg < wend) {
    // first slot: the largest s in [s_lo, s_hi) with wp[s] - W0 <= wbeg
    int64_t a = s_lo, b = s_hi;
    while (b - a > 1) {
      const int64_t mid = (a + b) >> 1;
      if (wp[mid] - W0 <= wbeg) a = mid; else b = mid;
    }
    int64_t sa = a;
    for (;;) {
      const int64_t sl = sa + ln;
      int32_t bu = 0, cu = 0, off = 0;
      int phu = 0;
      if (sl < s_hi) {
        const int64_t ws = wp[sl] - W0, we = wp[sl + 1] - W0;
        const int64_t lo = max(ws, wbeg), hi = min(we, wend);
        if (hi > lo) {
          const int32_t sx = bx + (int32_t)(sl - s_lo);
          bu = rp[ci[sx]];
          phu = (int)(cdt[sx] & 15u);
          cu = (int32_t)(hi - lo);
          off = (int32_t)(lo - ws);
        }
      }
      int32_t tot = 0;
      const int32_t excl = wave_excl_scan(cu, &tot);
      constexpr int U = 2;
      for (int32_t c0 = 0; c0 < tot; c0 += TG_WAVE * U) {
        int32_t wid[U], pv[U];
        uint32_t dt[U];
        bool ok[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int32_t v = c0 + j * TG_WAVE + ln;
          // owner lane: the largest l with excl[l] <= v
          int o = 0;
          for (int step = 32; step > 0; step >>= 1) {
            const int32_t ex = __shfl(excl, o + step, TG_WAVE);
            if (o + step < TG_WAVE && ex <= v) o += step;
          }
          const int32_t o_excl = __shfl(excl, o, TG_WAVE);
          const int32_t o_bu = __shfl(bu, o, TG_WAVE);
          const int32_t o_off = __shfl(off, o, TG_WAVE);
          pv[j] = __shfl(phu, o, TG_WAVE);
          ok[j] = v < tot;
          const int32_t sv = o_bu + o_off + (v - o_excl);
          wid[j] = ok[j] ? ci[sv] : 0;
          dt[j] = ok[j] ? cdt[sv] : 0u;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int32_t w = wid[j];
          if (!ok[j] || !precedes((int32_t)(dt[j] >> 4), w, dx, x)) continue;
          const uint32_t k = (uint32_t)w / (uint32_t)R;
          const uint32_t rank = atomicAdd(&hist[k], 1u);
          const uint32_t idx = atomicAdd(nst, 1u);
          srec[idx] = (((uint32_t)w - k * (uint32_t)R) << 4) | (uint32_t)pv[j];
          skey[idx] = (k << 16) | rank;
        }
      }
      // next window, unless it starts at or past this wavefront's last wedge
      sa += TG_WAVE;
      if (sa >= s_hi || wp[sa] - W0 >= wend) break;
    }
  }
  __syncthreads();
  // range starts: exclusive prefix of the histogram, by wavefront 0
  int32_t* myruns = runs + (int64_t)blockIdx.x * (K + 1);
  if (wv == 0) {
    int32_t carry = 0;
    for (int k0 = 0; k0 < K; k0 += TG_WAVE) {
      const int k = k0 + ln;
      const int32_t h = k < K ? (int32_t)hist[k] : 0;
      int32_t tot = 0;
      const int32_t ex = wave_excl_scan(h, &tot);
      if (k < K) {
        hist[k] = (uint32_t)(carry + ex);
        myruns[k] = carry + ex;
      }
      carry += tot;
    }
    if (ln == 0) myruns[K] = carry;
  }
  __syncthreads();
  const uint32_t ns = *nst;
  uint32_t* dst = region + (int64_t)blockIdx.x * CHW;
  for (uint32_t i = threadIdx.x; i < ns; i += blockDim.x) {
    const uint32_t key = skey[i];
    dst[hist[key >> 16] + (key & 0xffffu)] = srec[i];
  }
}

// LDS bytes of k_c4_bcount: the table, then per-thread run starts and the
// prefix of run lengths.
__host__ __device__ inline size_t c4_bcount_lds(int R, int RWp, int NT) {
  return (size_t)R * RWp * sizeof(uint32_t) + (size_t)NT * sizeof(int64_t) + (size_t)(NT + 1) * sizeof(int32_t);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_c4_bcount(int K, int R, int RWp, int64_t n,
                                                  const int32_t* __restrict__ nit,
                                                  const uint32_t* __restrict__ region, int CHW,
                                                  const int32_t* __restrict__ runs, uint32_t* __restrict__ out,
                                                  int64_t stride) {
  extern __shared__ uint4 bc_lds[];
  uint32_t* table = reinterpret_cast<uint32_t*>(bc_lds);
  const int tw = R * RWp;  // a multiple of 4
  int64_t* bst = reinterpret_cast<int64_t*>(table + tw);
  int32_t* bpre = reinterpret_cast<int32_t*>(bst + NT);
  const int gi = blockIdx.x / K, k = blockIdx.x % K;
  const int t = threadIdx.x;
  for (int i = t; i < tw / 4; i += NT) bc_lds[i] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  const int32_t i0 = nit[gi], i1 = nit[gi + 1];
  for (int32_t b0 = i0; b0 < i1; b0 += NT) {
    // this batch's runs of range k, one item per thread, and their prefix
    const int32_t itm = b0 + t;
    int32_t len = 0;
    if (itm < i1) {
      const int32_t r0 = runs[(int64_t)itm * (K + 1) + k], r1 = runs[(int64_t)itm * (K + 1) + k + 1];
      len = r1 - r0;
      bst[t] = (int64_t)itm * CHW + r0;
    }
    bpre[t + 1] = len;
    if (t == 0) bpre[0] = 0;
    __syncthreads();
    for (int d = 1; d < NT; d <<= 1) {
      const int32_t add = (t + 1 > d) ? bpre[t + 1 - d] : 0;
      __syncthreads();
      bpre[t + 1] += add;
      __syncthreads();
    }
    const int32_t total = bpre[NT];
    for (int32_t v = t; v < total; v += NT) {
      // owner: the largest s with bpre[s] <= v
      int s = 0;
      for (int step = NT / 2; step > 0; step >>= 1)
        if (bpre[s + step] <= v) s += step;
      const uint32_t rec = region[bst[s] + (v - bpre[s])];
      const uint32_t ph = rec & 15u;
      atomicAdd(&table[(rec >> 4) * RWp + (ph >> 1)], 1u << ((ph & 1u) << 4));
    }
    __syncthreads();
  }
  // the range's rows out, padded to 4 words: only the rows of far ends
  // that some wedge of the node reaches, the only rows the credit walk
  // reads (a row left alone may hold an earlier node's counts)
  const int64_t lo = (int64_t)k * R;
  const int32_t nr = (int32_t)(lo + R < n ? R : n - lo);
  uint4* dst = reinterpret_cast<uint4*>(out + (int64_t)gi * stride + lo * 4);
  for (int32_t r = t; r < nr; r += NT) {
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = j < RWp ? table[r * RWp + j] : 0u;
    if (v[0] | v[1] | v[2] | v[3]) dst[r] = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

}  // namespace tg
