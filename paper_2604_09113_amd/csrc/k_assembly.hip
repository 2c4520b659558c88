// Batched stiffness contraction (A3): for every cell
//   K[(i1,n1),(i2,n2)] = sum_s theta[i1 i2, s] * sum_r Uhat[(n1,n2,s), r] Itil[r]
// i.e. the reduced reconstruction I = Uhat Itil (Alg. 5) followed by the
// fast-assembly contraction with the geometry coefficients (Alg. 4), with the
// stabilisation folded in as the last column of Uhat = [U_r | I_pi].
//
// Only node pairs n2 <= n1 (permuted node order: interior, corners, edges) are
// formed, since K is symmetric.  The reconstruction is a real dense GEMM
// (rows = (pair, s), columns = cells, depth = n_r + 1 padded to 4*KC) and runs on
// MFMA 16x16x4 (FP64 for the operator, FP32 for the single-precision copy).  The
// 36 -> 4 contraction over s runs in the epilogue: a tile holds 16 pairs of one s
// for 16 cells, so each lane accumulates its pairs' 4 (i1, i2) entries over s in
// registers and no cross-lane reduction is needed.
//
// Workgroup: 4 waves x 32 cells on one 16-pair tile; consecutive workgroups
// walk the cells of one (family, cluster) group, so a pair tile of Uhat is
// streamed from L2 by every workgroup on an XCD at about the same time.
// The geometry coefficients are read from a copy in tile order
// ([tile][s][128 cells][4], k_theta_tile): the 16 cells of a block at one step
// are one contiguous 256 B (FP32) segment, where the cell-major array would
// touch 16 cache lines per load, re-read for every one of the ~208 pair tiles.
#include <cstdio>
#include <mutex>

#include "internal.h"

namespace lbddc {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T> struct V4;
template <> struct V4<double> { typedef dbl4 type; };
template <> struct V4<float> { typedef flt4 type; };

__device__ inline dbl4 mfma(double a, double b, dbl4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline flt4 mfma(float a, float b, flt4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// tiles[i] = {group, first position in `sorted`, number of cells, unused}
// theta_t[tile][s][o][e] = theta[sorted[start + o]][s][e] for the tile's
// cells o < count (TS cells per tile), zero for the unused slots of a partial tile
template <typename T, int TS>
__global__ __launch_bounds__(256) void k_theta_tile(const T* __restrict__ theta, const int* __restrict__ sorted,
                                                    const int4* __restrict__ tiles, int ns, T* __restrict__ theta_t) {
  typedef typename V4<T>::type v4;
  const int4 td = tiles[blockIdx.x];
  T* out = theta_t + (size_t)blockIdx.x * ns * TS * 4;
  for (int i = threadIdx.x; i < ns * TS; i += 256) {
    const int st = i / TS, o = i % TS;
    v4 v = v4{0, 0, 0, 0};
    if (o < td.z) v = *reinterpret_cast<const v4*>(theta + ((size_t)sorted[td.y + o] * ns + st) * 4);
    *reinterpret_cast<v4*>(out + (size_t)i * 4) = v;
  }
}

// the FP64 coefficients in the order of 16-cell tiles (the adjoint's tiles)
hipError_t launch_theta_tile16(Ctx* c, const int4* tiles, int ntiles, double* out) {
  if ((size_t)ntiles * 16 > (size_t)(c->ncell / 128 + 17) * 128) return hipErrorInvalidValue;  // buffer size
  hipLaunchKernelGGL((k_theta_tile<double, 16>), dim3(ntiles), dim3(256), 0, c->stream, c->d_theta, c->d_sorted,
                     tiles, c->ns, out);
  return hipGetLastError();
}

template <typename T, int KC>
__global__ __launch_bounds__(256) void k_assemble(const T* const* __restrict__ utg, const T* __restrict__ theta_t,
                                                  const T* __restrict__ itil, const int* __restrict__ sorted,
                                                  const int4* __restrict__ tiles, T* __restrict__ K, int ns,
                                                  int npair, int itil_stride) {
  typedef typename V4<T>::type v4;
  const int pt = blockIdx.y;
  const int4 td = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  int cidx[2];
  bool cval[2];
#pragma unroll
  for (int bk = 0; bk < 2; ++bk) {
    int o = wave * 32 + bk * 16 + col;
    cval[bk] = o < td.z;
    cidx[bk] = sorted[td.y + (cval[bk] ? o : 0)];
  }
  T b[2][KC];
#pragma unroll
  for (int bk = 0; bk < 2; ++bk)
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) b[bk][kc] = itil[(size_t)cidx[bk] * itil_stride + 4 * kc + grp];
  v4 acc[2][4];
#pragma unroll
  for (int bk = 0; bk < 2; ++bk)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[bk][e] = v4{0, 0, 0, 0};
  // The group's Uhat is read through a pointer loaded from memory: say that it
  // is global memory, so the loads are global loads (a flat load would also be
  // counted by the LDS/scalar counter, whose waits would then drain the
  // prefetch).  Two register sets take the steps of s in turn, each reloaded
  // (for s + 2) right after the step that used it, without copies between
  // them, so every load has a whole step of MFMA work to arrive.
  typedef const T __attribute__((address_space(1)))* GP;
  const GP ap = (GP)utg[td.x] + (size_t)pt * ns * KC * 64 + lane;
  const T* th0 = theta_t + ((size_t)blockIdx.x * ns * 128 + wave * 32 + col) * 4;
  const T* th1 = th0 + 16 * 4;
  T aA[KC], aB[KC];
  v4 tA0, tA1, tB0, tB1;
  auto load = [&](int sl, T (&a)[KC], v4& t0, v4& t1) {
    sl = sl < ns ? sl : ns - 1;  // past the end: a valid step, not used
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) a[kc] = ap[((size_t)sl * KC + kc) * 64];
    t0 = *reinterpret_cast<const v4*>(th0 + (size_t)sl * 512);
    t1 = *reinterpret_cast<const v4*>(th1 + (size_t)sl * 512);
  };
  auto step = [&](const T (&a)[KC], const v4& t0, const v4& t1) {
    v4 d0 = v4{0, 0, 0, 0}, d1 = v4{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      d0 = mfma(a[kc], b[0][kc], d0);
      d1 = mfma(a[kc], b[1][kc], d1);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[0][e] += t0[e] * d0;
      acc[1][e] += t1[e] * d1;
    }
  };
  load(0, aA, tA0, tA1);
  load(1, aB, tB0, tB1);
  for (int s = 0; s < ns; s += 2) {  // ns = 4 (q + 1)^2 is even
    step(aA, tA0, tA1);
    load(s + 2, aA, tA0, tA1);
    step(aB, tB0, tB1);
    load(s + 3, aB, tB0, tB1);
  }
  // lane (grp, col) holds pairs 4*grp + v of its cell
#pragma unroll
  for (int bk = 0; bk < 2; ++bk) {
    if (!cval[bk]) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int P = pt * 16 + 4 * grp + v;
      if (P < npair) {
        v4 o = v4{acc[bk][0][v], acc[bk][1][v], acc[bk][2][v], acc[bk][3][v]};
        *reinterpret_cast<v4*>(K + ((size_t)cidx[bk] * npair + P) * 4) = o;
      }
    }
  }
}

// Stable counting sort of the cells by group (one workgroup of 1024 threads,
// G <= 16 groups): thread t takes cells [t c, t c + c), counts them per group
// in registers, and the per-group exclusive prefix over the threads (a wave
// scan by shuffles, then the wave totals) gives each thread its write
// positions; within a thread the cells keep their order.  Deterministic.
constexpr int kSortT = 1024;
__global__ __launch_bounds__(kSortT) void k_group_sort(const int* __restrict__ group, int ncell, int G,
                                                       int* __restrict__ sorted, int* __restrict__ counts) {
  __shared__ int wtot[16][kSortT / 64];  // per group, per wave: the wave's count
  __shared__ int gbase[17];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int chunk = (ncell + kSortT - 1) / kSortT;
  const int b0 = min(ncell, t * chunk), b1 = min(ncell, b0 + chunk);
  int cnt[16];
#pragma unroll
  for (int g = 0; g < 16; ++g) cnt[g] = 0;
  for (int i = b0; i < b1; ++i) {
    int g = group[i];
    g = g < 0 ? 0 : (g >= G ? G - 1 : g);
#pragma unroll
    for (int q = 0; q < 16; ++q) cnt[q] += g == q;
  }
  // inclusive wave scan of each group's counts, then the exclusive offset
  int off[16];
#pragma unroll
  for (int g = 0; g < 16; ++g) {
    int v = cnt[g];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    off[g] = v - cnt[g];
    if (lane == 63) wtot[g][wave] = v;
  }
  __syncthreads();
  if (t < 16) {  // thread g: prefix over the waves of group g, and the group total
    int run = 0;
    for (int w = 0; w < kSortT / 64; ++w) {
      const int c = wtot[t][w];
      wtot[t][w] = run;
      run += c;
    }
    gbase[t + 1] = run;
  }
  __syncthreads();
  if (t == 0) {
    gbase[0] = 0;
    for (int g = 0; g < 16; ++g) {
      if (g < G) counts[g] = gbase[g + 1];
      gbase[g + 1] += gbase[g];
    }
  }
  __syncthreads();
  int pos[16];
#pragma unroll
  for (int g = 0; g < 16; ++g) pos[g] = gbase[g] + wtot[g][wave] + off[g];
  for (int i = b0; i < b1; ++i) {
    int g = group[i];
    g = g < 0 ? 0 : (g >= G ? G - 1 : g);
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (g == q) sorted[pos[q]++] = i;
  }
}

template <typename T>
static hipError_t launch_family(Ctx* c, const T* const* d_utg, int KC, const T* theta, const T* itil,
                                const int4* tiles, int ntiles, T* K) {
  dim3 grid(ntiles, c->NPT), block(256);
  const int st = 4 * c->KC;
  if (c->ns % 2 != 0) return hipErrorInvalidValue;  // the kernel takes the steps of s in pairs
#define LB_CASE(kc)                                                                                       \
  case kc:                                                                                                \
    hipLaunchKernelGGL((k_assemble<T, kc>), grid, block, 0, c->stream, d_utg, theta, itil, c->d_sorted, \
                       tiles, K, c->ns, c->npair, st);                                                  \
    break;
  switch (KC) {
    LB_CASE(1) LB_CASE(2) LB_CASE(3) LB_CASE(4) LB_CASE(5) LB_CASE(6) LB_CASE(7) LB_CASE(8) LB_CASE(9)
    LB_CASE(10) LB_CASE(11)
    default: return hipErrorInvalidValue;
  }
#undef LB_CASE
  return hipGetLastError();
}

// Buffers of one contraction: the tile table (int4 per tile), the per-group
// Uhat pointers (16), the tile-ordered geometry coefficients of the precision
// used (room for `theta_tiles` tiles) and the output K.
struct AsmBuffers {
  int* tiles;
  void** ptrs;
  void* theta_t;
  size_t theta_tiles;
  void* K;
  bool cacheable;  // the tile table and pointers stay in place between calls
};

static hipError_t launch_assembly_into(Ctx* c, bool fp32, const AsmBuffers& bf, hipEvent_t e0, hipEvent_t e1) {
  // groups: family slot s owns groups [base_s, base_s + n_cl)
  int G = 0;
  std::vector<int> base;
  for (int fid : c->fam_ids) {
    base.push_back(G);
    G += c->roms[fid].ncl;
  }
  if (G > 16) return hipErrorInvalidValue;
  Ctx::GroupCache& gc = c->grp;
  const bool reuse = bf.cacheable && gc.gen == c->geom_gen && gc.fp32 == fp32 && gc.tiles == bf.tiles;
  std::vector<int> fam_first, fam_n;
  hipError_t e = hipSuccess;
  if (reuse) {
    fam_first = gc.fam_first;
    fam_n = gc.fam_n;
    c->ntiles = gc.ntiles;
  } else {
  int* d_counts = c->d_flags + 8 + 64;
  hipLaunchKernelGGL(k_group_sort, dim3(1), dim3(kSortT), 0, c->stream, c->d_cluster, c->ncell, G, c->d_sorted, d_counts);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int counts[16];
  e = hipMemcpyAsync(c->h_flags + 8, d_counts, G * sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  for (int g = 0; g < G; ++g) counts[g] = c->h_flags[8 + g];
  c->group_counts.assign(counts, counts + G);
  // tiles of 128 cells per group, per family
  std::vector<int> tiles;
  int start = 0;
  c->group_family.assign(G, 0);
  c->group_cluster.assign(G, 0);
  for (size_t s = 0; s < c->fam_ids.size(); ++s) {
    fam_first.push_back((int)tiles.size() / 4);
    for (int k = 0; k < c->roms[c->fam_ids[s]].ncl; ++k) {
      int g = base[s] + k;
      c->group_family[g] = (int)s;
      c->group_cluster[g] = k;
      for (int o = 0; o < counts[g]; o += 128) {
        tiles.push_back(g);
        tiles.push_back(start + o);
        tiles.push_back(std::min(128, counts[g] - o));
        tiles.push_back(0);
      }
      start += counts[g];
    }
    fam_n.push_back((int)tiles.size() / 4 - fam_first.back());
  }
  c->ntiles = (int)tiles.size() / 4;
  if ((size_t)c->ntiles > bf.theta_tiles) return hipErrorInvalidValue;  // size of the tile-ordered theta
  // tile table and per-group Uhat pointers
  std::vector<const void*> ptrs(G, nullptr);
  for (int g = 0; g < G; ++g) {
    const RomDev& R = c->roms[c->fam_ids[c->group_family[g]]];
    ptrs[g] = fp32 ? (const void*)R.ut32[c->group_cluster[g]] : (const void*)R.ut64[c->group_cluster[g]];
  }
  e = hipMemcpyAsync(bf.tiles, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(bf.ptrs, ptrs.data(), G * sizeof(void*), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  if (bf.cacheable) {
    gc.gen = c->geom_gen;
    gc.fp32 = fp32;
    gc.tiles = bf.tiles;
    gc.ntiles = c->ntiles;
    gc.fam_first = fam_first;
    gc.fam_n = fam_n;
  } else {
    gc.gen = 0;
  }
  }
  c->tile_fam_first = fam_first;
  c->tile_fam_n = fam_n;
  // the reduced coordinates of the four-parameter families, on the same tiles
  for (size_t s = 0; s < c->fam_ids.size(); ++s) {
    e = launch_mdeim4(c, (int)s, bf.tiles, fam_first[s], fam_n[s]);
    if (e != hipSuccess) return e;
  }
  if (e0) hipEventRecord(e0, c->stream);
  const int4* d_tl = reinterpret_cast<const int4*>(bf.tiles);
  if (fp32)
    hipLaunchKernelGGL((k_theta_tile<float, 128>), dim3(c->ntiles), dim3(256), 0, c->stream, c->d_theta32, c->d_sorted, d_tl,
                       c->ns, (float*)bf.theta_t);
  else
    hipLaunchKernelGGL((k_theta_tile<double, 128>), dim3(c->ntiles), dim3(256), 0, c->stream, c->d_theta, c->d_sorted, d_tl,
                       c->ns, (double*)bf.theta_t);
  for (size_t s = 0; s < c->fam_ids.size(); ++s) {
    if (fam_n[s] == 0) continue;
    const int4* tl = d_tl + fam_first[s];
    const size_t toff = (size_t)fam_first[s] * c->ns * 512;
    const int KC = c->roms[c->fam_ids[s]].KC;
    if (fp32)
      e = launch_family<float>(c, (const float* const*)bf.ptrs, KC, (const float*)bf.theta_t + toff, c->d_itil32, tl,
                               fam_n[s], (float*)bf.K);
    else
      e = launch_family<double>(c, (const double* const*)bf.ptrs, KC, (const double*)bf.theta_t + toff, c->d_itil, tl,
                                fam_n[s], (double*)bf.K);
    if (e != hipSuccess) return e;
  }
  if (e1) hipEventRecord(e1, c->stream);
  return hipGetLastError();
}

hipError_t launch_assembly(Ctx* c, bool fp32, hipEvent_t e0, hipEvent_t e1) {
  AsmBuffers bf;
  bf.tiles = c->d_tiles;
  bf.ptrs = (void**)(c->d_tiles + 4 * (c->ncell / 16 + 64));  // after the tile table, sized for 16 groups
  bf.theta_t = fp32 ? (void*)c->d_theta_t32 : (void*)c->d_theta_t;
  bf.theta_tiles = (size_t)c->ncell / 128 + 17;
  bf.K = fp32 ? (void*)c->d_K32 : (void*)c->d_K;
  bf.cacheable = true;
  return launch_assembly_into(c, fp32, bf, e0, e1);
}

// ---------------------------------------------------------------------------
// Staging of lbddc_assemble_fp32_noalloc, a static device array: the tile
// table, the per-group Uhat pointers and the tile-ordered FP32 geometry
// coefficients.  Each GPU the library runs on holds its own copy until the
// process ends; host code reaches it only through the address taken with
// hipGetSymbolAddress (per device, at lbddc_create), never through the name.
// Every call on one GPU shares it: calls that overlap on a GPU race.
constexpr size_t kScratchTableBytes = 64u << 10;   // tile table, up to 4096 tiles
constexpr size_t kScratchPtrBytes = 64u << 10;     // per-group Uhat pointers (16 used)
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static void* g_scratch_addr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[device] = ptr;
  return hipSuccess;
}

lbddc_status assemble_fp32_noalloc(Ctx* c, float* d_K) {
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) base = g_scratch_addr[c->device];
  }
  if (!base) {
    c->err = "assemble_fp32_noalloc: the static scratch of this device has no address";
    return LBDDC_E_HIP;
  }
  // the tile-ordered coefficients take ns * 128 * 4 floats per tile of 128
  // cells of one group; the tile count is known exactly after the group sort
  // (at most one partial tile per group more than ncell / 128)
  const size_t per_tile = (size_t)c->ns * 128 * 4 * sizeof(float);
  const size_t cap = std::min((kNoAllocScratchBytes - kScratchTableBytes - kScratchPtrBytes) / per_tile,
                              kScratchTableBytes / (4 * sizeof(int)));
  auto too_large = [&](size_t ntiles) {
    char buf[240];
    snprintf(buf, sizeof buf,
             "assemble_fp32_noalloc: %d cells take %zu tiles of 128 cells, more than the %zu that the %zu-byte static "
             "scratch holds at (q+1)^2 = %d",
             c->ncell, ntiles, cap, kNoAllocScratchBytes, c->nL);
    c->err = buf;
    return LBDDC_E_UNSUPPORTED;
  };
  if (((size_t)c->ncell + 127) / 128 > cap) return too_large(((size_t)c->ncell + 127) / 128);
  hipError_t e = launch_geometry(c);
  if (e == hipSuccess) {
    AsmBuffers bf;
    bf.tiles = (int*)base;
    bf.ptrs = (void**)((char*)base + kScratchTableBytes);
    bf.theta_t = (char*)base + kScratchTableBytes + kScratchPtrBytes;
    bf.theta_tiles = cap;
    bf.K = d_K;
    bf.cacheable = false;  // the staging array is shared by every call on this GPU
    e = launch_assembly_into(c, true, bf, nullptr, nullptr);
    if (e == hipErrorInvalidValue && (size_t)c->ntiles > cap) return too_large(c->ntiles);
  }
  if (e != hipSuccess) {
    c->err = std::string("assemble_fp32_noalloc: ") + hipGetErrorString(e);
    return LBDDC_E_HIP;
  }
  return LBDDC_OK;
}

}  // namespace lbddc
