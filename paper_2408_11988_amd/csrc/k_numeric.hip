// Numeric phase of row-wise Gustavson TS-SpGEMM (Sec. III-A, Eq. 1):
// C(i,:) = sum over k in pat(A_i) of A(i,k) B(k,:), with the dense accumulator
// (SPA) of width d that Sec. III-C prefers for d <= 1024. On gfx950 a strip of
// d accumulators lives in LDS (FP64 for the FP32 semiring: every FP32 x FP32
// product is exact in FP64 and is added with the native ds_add_f64, then
// rounded once to FP32 at the end).
//
// The kernel is bound by the latency of dependent gathers (A entry -> B row
// pointers -> B row), so the work layout is about keeping many rows in flight.
// Rows are binned by their product count flops_i (Sec. II-A):
//  * light rows: a group of GL lanes owns one row and one strip, so 256/GL
//    rows per workgroup are in flight; groups walk the binned list with a
//    grid stride, so neighbouring groups get rows of similar cost;
//  * wavefront rows: one wavefront per row, four rows per workgroup;
//  * workgroup rows: the four wavefronts of a workgroup share the row, each
//    accumulating a private strip, summed in a fixed order;
//  * split rows: chunks of A entries go to separate workgroups, each writes
//    its partial strip to global memory; a second kernel adds the partials in
//    chunk order and writes the row.
// Every order of addition is fixed, so results are reproducible run to run.
// Streaming B: a group of GL lanes reads one B row (GL consecutive entries per
// step, coalesced); several A entries are unrolled so that several B rows are
// in flight per group.
// Output: the row's pattern is already known as a bitmap (symbolic phase);
// a lane owns column j of a chunk, and its output slot is the popcount of the
// set bits below it, so columns come out sorted without a sort.
#include "dev_numeric.hpp"

namespace tss {

template <int GL, typename T, typename BR, int LAYOUT>
__global__ __launch_bounds__(kBlock) void k_numeric(NumParams np) {
  using S = SemiringT<T>;
  using Acc = typename S::acc;
  extern __shared__ __align__(16) unsigned char smem[];
  const Problem& pr = np.pr;
  const int d = pr.d;
  Acc* strips = (Acc*)smem;
  int4* stage = (int4*)(smem + (size_t)kWavesPerBlock * d * sizeof(Acc));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int g = blockIdx.x;
  const bool wg_mode = g < np.n_wg_items;
  Item it{-1, 0, 0, 0};
  bool valid;
  if (wg_mode) {
    it = np.items[g];
    valid = true;
  } else {
    const int64_t idx = (int64_t)np.n_wg_items + 4 * (int64_t)(g - np.n_wg_items) + wave;
    valid = idx < np.n_heavy_records;
    if (valid) it = np.items[idx];
  }
  Acc* strip = strips + wave * d;
  for (int j = lane; j < d; j += kWave) strip[j] = Acc(0);
  __syncthreads();
  if (valid) {
    if (wg_mode)
      accumulate_range<GL, T, BR, LAYOUT>(pr, it.p0, it.p1, wave, kWavesPerBlock, strip, stage + wave * kWave);
    else
      accumulate_range<GL, T, BR, LAYOUT>(pr, it.p0, it.p1, 0, 1, strip, stage + wave * kWave);
  }
  __syncthreads();
  if (wg_mode) {
    for (int j = threadIdx.x; j < d; j += kBlock)
      strips[j] = S::add(S::add(S::add(strips[j], strips[d + j]), strips[2 * d + j]), strips[3 * d + j]);
    __syncthreads();
    if (it.aux != kNoSlot) {
      // split chunk: partial sums to its slot (added up by k_split_finalize)
      if constexpr (sizeof(Acc) == 8) {
        double* dst = np.partial + (int64_t)it.aux * d;
        for (int j = threadIdx.x; j < d; j += kBlock) dst[j] = strips[j];
      } else {
        int32_t* dst = np.ipartial + (int64_t)it.aux * d;
        for (int j = threadIdx.x; j < d; j += kBlock) dst[j] = strips[j];
      }
    } else {
      emit_row<T>(pr, it.row, strips, wave, kWavesPerBlock);
    }
  } else if (valid) {
    emit_row<T>(pr, it.row, strip, 0, 1);
  }
}

template <int GL, typename T, typename BR, int LAYOUT>
__global__ __launch_bounds__(kBlock) void k_numeric_light(NumParams np) {
  using Acc = typename SemiringT<T>::acc;
  constexpr int G = kBlock / GL;  // rows in flight per workgroup
  extern __shared__ __align__(16) unsigned char smem[];
  const Problem& pr = np.pr;
  const int d = pr.d;
  const int grp = threadIdx.x / GL, gl = threadIdx.x % GL;
  Acc* strip = (Acc*)smem + grp * d;
  int4* stage = (int4*)(smem + (size_t)G * d * sizeof(Acc)) + grp * GL;
  const Item* items = np.items + np.n_heavy_records;
  const int64_t stride = (int64_t)gridDim.x * G;
  for (int64_t t = (int64_t)blockIdx.x * G + grp; t < np.n_light; t += stride) {
    const Item it = items[t];
    for (int j = gl; j < d; j += GL) strip[j] = Acc(0);
    wave_sync();
    accumulate_light<GL, T, BR, LAYOUT>(pr, it.p0, it.p1, strip, stage, gl);
    wave_sync();
    emit_group<GL, T>(pr, it.row, strip, gl);
    wave_sync();
  }
}

// ---------------------------------------------------------------- launch

static size_t acc_bytes(int sr) { return sr == TSSPGEMM_PLUS_TIMES_F32 ? 8 : 4; }

int light_group_lanes(int group_lanes, int64_t d, int sr) {
  // strips of all groups of a workgroup within 16 KB of LDS, so that eight
  // workgroups (32 wavefronts) fit a CU: wide strips take wider groups
  int gl = group_lanes;
  while (gl < 64 && (size_t)(kBlock / gl) * d * acc_bytes(sr) > 16384) gl <<= 1;
  return gl;
}

static int64_t light_grid(int64_t n_light, int gl) {
  const int64_t per_block = kBlock / gl;
  int64_t g = (n_light + per_block - 1) / per_block;
  const int64_t cap = 256 * 8;  // CUs x resident workgroups
  return g < cap ? g : cap;
}

int col_id_bytes(int64_t d) { return d <= 256 ? 1 : 2; }

template <typename T, typename BR, int LAYOUT>
static int launch_numeric_t(int group_lanes, const NumParams& np, int64_t n_grid, hipStream_t st) {
  const size_t ab = sizeof(typename SemiringT<T>::acc);
  if (n_grid > 0) {
    const size_t lds = (size_t)kWavesPerBlock * np.pr.d * ab + kWavesPerBlock * kWave * sizeof(int4);
    switch (LAYOUT == kLayoutFlat ? 64 : group_lanes) {  // the flat layout uses the whole wavefront
      case 4: k_numeric<4, T, BR, LAYOUT><<<(unsigned)n_grid, kBlock, lds, st>>>(np); break;
      case 8: k_numeric<8, T, BR, LAYOUT><<<(unsigned)n_grid, kBlock, lds, st>>>(np); break;
      case 16: k_numeric<16, T, BR, LAYOUT><<<(unsigned)n_grid, kBlock, lds, st>>>(np); break;
      case 32: k_numeric<32, T, BR, LAYOUT><<<(unsigned)n_grid, kBlock, lds, st>>>(np); break;
      case 64: k_numeric<64, T, BR, LAYOUT><<<(unsigned)n_grid, kBlock, lds, st>>>(np); break;
      default:
        set_error("numeric: group_lanes must be 4, 8, 16, 32 or 64");
        return TSSPGEMM_ERR_INVALID_ARG;
    }
    TSS_CHECK_LAUNCH();
  }
  if (np.n_light > 0) {
    const int gl = light_group_lanes(group_lanes, np.pr.d, sizeof(typename SemiringT<T>::acc) == 8
                                                               ? TSSPGEMM_PLUS_TIMES_F32 : TSSPGEMM_PLUS_TIMES_I32);
    const unsigned g = (unsigned)light_grid(np.n_light, gl);
    const size_t lds = (size_t)(kBlock / gl) * np.pr.d * ab + kBlock * sizeof(int4);
    switch (gl) {
      case 4: k_numeric_light<4, T, BR, LAYOUT><<<g, kBlock, lds, st>>>(np); break;
      case 8: k_numeric_light<8, T, BR, LAYOUT><<<g, kBlock, lds, st>>>(np); break;
      case 16: k_numeric_light<16, T, BR, LAYOUT><<<g, kBlock, lds, st>>>(np); break;
      case 32: k_numeric_light<32, T, BR, LAYOUT><<<g, kBlock, lds, st>>>(np); break;
      case 64: k_numeric_light<64, T, BR, LAYOUT><<<g, kBlock, lds, st>>>(np); break;
      default:
        set_error("numeric: bad light group width");
        return TSSPGEMM_ERR_INVALID_ARG;
    }
    TSS_CHECK_LAUNCH();
  }
  return TSSPGEMM_OK;
}

template <typename T, typename BR>
static int launch_numeric_l(int group_lanes, int products, const NumParams& np, int64_t n_grid, hipStream_t st) {
  switch (products) {
    case TSSPGEMM_PRODUCTS_FLAT: return launch_numeric_t<T, BR, kLayoutFlat>(group_lanes, np, n_grid, st);
    case TSSPGEMM_PRODUCTS_VEC4: return launch_numeric_t<T, BR, kLayoutVec>(group_lanes, np, n_grid, st);
    default: return launch_numeric_t<T, BR, kLayoutRows>(group_lanes, np, n_grid, st);
  }
}

// B's column ids are read narrowed (np.pr.bcol, col_id_bytes(d) bytes each).
// products: tsspgemm_products (resolved, not AUTO).
int launch_numeric(int sr, int group_lanes, int products, const NumParams& np, int64_t n_grid, hipStream_t st) {
  const bool b8 = col_id_bytes(np.pr.d) == 1;
  if (!np.pr.bcol && np.pr.n > 0) {
    set_error("numeric: narrowed column ids missing");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (sr == TSSPGEMM_PLUS_TIMES_F32)
    return b8 ? launch_numeric_l<float, BSep<uint8_t>>(group_lanes, products, np, n_grid, st)
              : launch_numeric_l<float, BSep<uint16_t>>(group_lanes, products, np, n_grid, st);
  return b8 ? launch_numeric_l<int32_t, BSep<uint8_t>>(group_lanes, products, np, n_grid, st)
            : launch_numeric_l<int32_t, BSep<uint16_t>>(group_lanes, products, np, n_grid, st);
}

// Split rows: add the chunks' partial strips in chunk order, then emit.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_split_finalize(Problem pr, const SplitRow* rows, const double* partial,
                                                           const int32_t* ipartial) {
  using S = SemiringT<T>;
  using Acc = typename S::acc;
  extern __shared__ __align__(16) unsigned char smem[];
  Acc* strip = (Acc*)smem;
  const SplitRow r = rows[blockIdx.x];
  const int d = pr.d;
  for (int j = threadIdx.x; j < d; j += kBlock) {
    Acc s = Acc(0);
    for (int c = 0; c < r.count; ++c) {
      if constexpr (sizeof(Acc) == 8)
        s = S::add(s, partial[(int64_t)(r.first + c) * d + j]);
      else
        s = S::add(s, ipartial[(int64_t)(r.first + c) * d + j]);
    }
    strip[j] = s;
  }
  __syncthreads();
  emit_row<T>(pr, r.row, strip, threadIdx.x >> 6, kWavesPerBlock);
}

int launch_split_finalize(int sr, const Problem& pr, const SplitRow* rows, int32_t nrows, const double* partial,
                          const int32_t* ipartial, hipStream_t st) {
  if (nrows == 0) return TSSPGEMM_OK;
  if (sr == TSSPGEMM_PLUS_TIMES_F32)
    k_split_finalize<float><<<nrows, kBlock, (size_t)pr.d * 8, st>>>(pr, rows, partial, ipartial);
  else
    k_split_finalize<int32_t><<<nrows, kBlock, (size_t)pr.d * 4, st>>>(pr, rows, partial, ipartial);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// (AND, OR): the output is the pattern alone. Lane = (row, word): each lane
// writes the set bits of one bitmap word, at the row start plus the popcount
// of the row's earlier words (segmented scan over the row's wp lanes).
__global__ void k_emit_pattern(Problem pr) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int wp = pr.wp;
  const int64_t row = t / wp;
  const int w = (int)(t % wp);
  const bool ok = row < pr.n;
  uint32_t word = ok ? pr.cbits[row * wp + w] : 0u;
  const int c = __popc(word);
  int x = c;
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < wp; o <<= 1) {
    const int y = __shfl_up(x, o, kWave);
    if ((lane % wp) >= o) x += y;
  }
  if (!ok || word == 0u) return;
  int pos = pr.crp[row] + x - c;
  while (word) {
    const int b = __ffs(word) - 1;
    pr.cci[pos++] = 32 * w + b;
    word &= word - 1;
  }
}

int launch_emit_pattern(const Problem& pr, hipStream_t st) {
  const int64_t lanes = (int64_t)pr.n * pr.wp;
  if (lanes == 0) return TSSPGEMM_OK;
  k_emit_pattern<<<grid_for(lanes, 256), 256, 0, st>>>(pr);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}


}  // namespace tss
