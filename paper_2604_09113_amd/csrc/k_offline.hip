// Offline stage of the method on the GPU (Sec. 4.2, Alg. 3): the snapshot
// integrals of the cells trimmed by the level sets of Table 1 with the
// bilinear threshold (Sec. 2.1.2), for thousands of parameter vectors at once.
//
//  k_rules        one thread per parameter vector: the implicit-domain
//                 quadrature rule of the trimmed cell (implicit_rule.h) into
//                 that vector's slot of the point buffers
//  k_snap_tensor  the whole trimmed tensor I[k1][k2][j1][j2][k3] =
//                 sum_points w dB_{k1,j1} dB_{k2,j2} L_k3 of one rule, a
//                 workgroup per (rule, k1), a thread per k2 <= k1 (the entry
//                 (k2, k1, j2, j1) is the same sum), the points staged in LDS
//                 64 at a time with their 1-D GLL bases and w L_k3
//  k_rule_entries selected entries of I (the magic points of the fitting
//                 stage): one thread per parameter vector generates its rule
//                 and adds each point's contribution to every selected entry
//                 as the point is produced, so no point is stored
//
// Results are deterministic: each rule's points are generated in a fixed
// order by one thread and every sum runs over them in that order.
#include "internal.h"
#include "implicit_rule.h"

namespace lbddc {

__global__ __launch_bounds__(64) void k_rules(const double* __restrict__ mu, int fam, int count, rule::Cfg g,
                                              double* px, double* py, double* pw, int cap, int* npts, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  rule::Cell c;
  c.fam = fam;
  for (int k = 0; k < 4; ++k) c.mu[k] = mu[(size_t)i * 4 + k];
  rule::Out o{px + (size_t)i * cap, py + (size_t)i * cap, pw + (size_t)i * cap, cap, 0, 0};
  rule::cell_rule(c, g, o);
  npts[i] = o.n;
  err[i] = o.err;
}

// Lagrange basis on `nodes` (n of them) at x: values v[a] and derivatives d[a]
__device__ inline void lagrange_vd(const double* nodes, int n, double x, double* v, double* d) {
  for (int a = 0; a < n; ++a) {
    double val = 1.0, der = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == a) continue;
      const double inv = 1.0 / (nodes[a] - nodes[l]);
      der = der * (x - nodes[l]) * inv + val * inv;  // product rule, one factor at a time
      val *= (x - nodes[l]) * inv;
    }
    v[a] = val;
    d[a] = der;
  }
}

struct SnapArgs {
  const double* px; const double* py; const double* pw; const int* npts; int cap;
  int p, q, nB, nL;
  const double* nodes;   // p+1 GLL nodes on [0, 1]
  const double* qnodes;  // q+1 GLL nodes
  double* out;           // [rule][n_i]
  long long n_i;
};

constexpr int kSnapCh = 64;

__global__ __launch_bounds__(128) void k_snap_tensor(SnapArgs g) {
  const int rule = blockIdx.y, k1 = blockIdx.x, k2 = threadIdx.x, t = threadIdx.x;
  const int P1 = g.p + 1, Q1 = g.q + 1, nL = g.nL;
  __shared__ double bx[kSnapCh][9], dbx[kSnapCh][9], by[kSnapCh][9], dby[kSnapCh][9], wl[kSnapCh][16];
  __shared__ double nd[9], qn[4];
  if (t < P1) nd[t] = g.nodes[t];
  if (t < Q1) qn[t] = g.qnodes[t];
  const int a1 = k1 % P1, b1 = k1 / P1, a2 = k2 % P1, b2 = k2 / P1;
  const bool active = k2 <= k1;
  double acc[4][16];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int k3 = 0; k3 < 16; ++k3) acc[j][k3] = 0.0;
  const int n = g.npts[rule];
  const double* X = g.px + (size_t)rule * g.cap;
  const double* Y = g.py + (size_t)rule * g.cap;
  const double* Wt = g.pw + (size_t)rule * g.cap;
  for (int c0 = 0; c0 < n; c0 += kSnapCh) {
    __syncthreads();
    if (t < kSnapCh && c0 + t < n) {
      const double x = X[c0 + t], y = Y[c0 + t], w = Wt[c0 + t];
      lagrange_vd(nd, P1, x, bx[t], dbx[t]);
      lagrange_vd(nd, P1, y, by[t], dby[t]);
      double lx[4], ly[4], dd[4];
      lagrange_vd(qn, Q1, x, lx, dd);
      lagrange_vd(qn, Q1, y, ly, dd);
      for (int b = 0; b < Q1; ++b)
        for (int a = 0; a < Q1; ++a) wl[t][a + Q1 * b] = w * lx[a] * ly[b];
    }
    __syncthreads();
    if (!active) continue;
    const int m = min(kSnapCh, n - c0);
    for (int i = 0; i < m; ++i) {
      const double d10 = dbx[i][a1] * by[i][b1], d11 = bx[i][a1] * dby[i][b1];
      const double d20 = dbx[i][a2] * by[i][b2], d21 = bx[i][a2] * dby[i][b2];
      const double pr[4] = {d10 * d20, d10 * d21, d11 * d20, d11 * d21};
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k3 = 0; k3 < 16; ++k3)
          if (k3 < nL) acc[j][k3] += pr[j] * wl[i][k3];
    }
  }
  if (!active) return;
  double* o = g.out + (size_t)rule * g.n_i;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int j1 = j >> 1, j2 = j & 1;
    for (int k3 = 0; k3 < nL; ++k3) {
      o[(((size_t)k1 * g.nB + k2) * 4 + j1 * 2 + j2) * nL + k3] = acc[j][k3];
      if (k1 != k2) o[(((size_t)k2 * g.nB + k1) * 4 + j2 * 2 + j1) * nL + k3] = acc[j][k3];
    }
  }
}

constexpr int kMaxEntries = 48;

// The entries sink: entry e is (k1, k2, j1, j2, k3) with k1 = a1 + (p+1) b1,
// k2 = a2 + (p+1) b2, k3 = a3 + (q+1) b3, decoded as dec[8 e ..] = {a1, b1,
// j1, a2, b2, j2, a3, b3}.
struct EntrySink {
  int ne, P1, Q1;
  const int* dec;
  const double* nodes;
  const double* qnodes;
  int err;
  double acc[kMaxEntries];
  __device__ void emit(double x, double y, double w) {
    double vx[9], dx[9], vy[9], dy[9], lx[4], ly[4], dq[4];
    lagrange_vd(nodes, P1, x, vx, dx);
    lagrange_vd(nodes, P1, y, vy, dy);
    lagrange_vd(qnodes, Q1, x, lx, dq);
    lagrange_vd(qnodes, Q1, y, ly, dq);
    for (int e = 0; e < ne; ++e) {
      const int* d = dec + 8 * e;
      const double g1 = d[2] == 0 ? dx[d[0]] * vy[d[1]] : vx[d[0]] * dy[d[1]];
      const double g2 = d[5] == 0 ? dx[d[3]] * vy[d[4]] : vx[d[3]] * dy[d[4]];
      acc[e] += w * (lx[d[6]] * ly[d[7]]) * g1 * g2;
    }
  }
};

__global__ __launch_bounds__(64) void k_rule_entries(const double* __restrict__ mu, int fam, int count, rule::Cfg g,
                                                     int p, int q, const double* nodes, const double* qnodes,
                                                     const int* dec, int ne, int dec_stride, double* out, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  rule::Cell c;
  c.fam = fam;
  for (int k = 0; k < 4; ++k) c.mu[k] = mu[(size_t)i * 4 + k];
  EntrySink s;
  s.ne = ne; s.P1 = p + 1; s.Q1 = q + 1; s.dec = dec + (size_t)i * dec_stride; s.nodes = nodes; s.qnodes = qnodes;
  s.err = 0;
  for (int e = 0; e < kMaxEntries; ++e) s.acc[e] = 0.0;
  rule::cell_rule(c, g, s);
  for (int e = 0; e < ne; ++e) out[(size_t)i * ne + e] = s.acc[e];
  err[i] = s.err;
}

}  // namespace lbddc

using namespace lbddc;

static lbddc_status off_fail(Ctx* c, lbddc_status s, const std::string& msg) {
  c->err = msg;
  return s;
}

// Gauss points per segment of the offline rules: exact along every segment
// (the integrand has degree <= 2p + q per variable) with margin across them.
static int offline_rule_points(int p, int q) { return std::max(12, p + q + 2); }

extern "C" lbddc_status lbddc_implicit_tensors(lbddc_ctx* x, int32_t family, int32_t p, int32_t q, int32_t count,
                                               const double* mu, int32_t n_entries, const int64_t* entries,
                                               int32_t entries_per_rule, double* out) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (family < 2 || family > 5) return off_fail(c, LBDDC_E_ARG, "implicit_tensors: family must be 2..5 (Table 1)");
  if (p < 2 || p > 8 || q < 1 || q > 3) return off_fail(c, LBDDC_E_UNSUPPORTED, "implicit_tensors: 2 <= p <= 8, 1 <= q <= 3");
  if (count < 0 || n_entries < 0 || n_entries > kMaxEntries || (count > 0 && (!mu || !out)) ||
      (n_entries > 0 && !entries))
    return off_fail(c, LBDDC_E_ARG, "implicit_tensors: bad sizes (at most 48 entries) or null pointers");
  if (count == 0) return LBDDC_OK;
  for (size_t i = 0; i < (size_t)count * 4; ++i)
    if (!std::isfinite(mu[i])) return off_fail(c, LBDDC_E_ARG, "implicit_tensors: non-finite threshold");
  const int nB = (p + 1) * (p + 1), nL = (q + 1) * (q + 1);
  const long long n_i = (long long)nB * nB * 4 * nL;
  const size_t n_ent_all = (size_t)n_entries * (entries_per_rule ? count : 1);
  for (size_t e = 0; e < n_ent_all; ++e)
    if (entries[e] < 0 || entries[e] >= n_i) return off_fail(c, LBDDC_E_ARG, "implicit_tensors: entry index out of range");
  hipSetDevice(c->device);
  const int n = offline_rule_points(p, q);
  std::vector<double> gx, gw;
  gauss_rule(n, gx, gw);
  const std::vector<double> nodes = gll_points(p), qnodes = gll_points(q);
  // whole tensors: rules into point buffers, 512 at a time; entries: 65536
  // rules at a time, each thread summing its entries as it makes its points
  const int cap = 1 << 17;
  const bool ent_mode = n_entries > 0;
  const int batch = ent_mode ? 65536 : 512;
  const size_t nout = ent_mode ? (size_t)n_entries : (size_t)n_i;
  double *d_g = nullptr, *d_mu = nullptr, *d_px = nullptr, *d_py = nullptr, *d_pw = nullptr, *d_out = nullptr;
  int *d_np = nullptr, *d_err = nullptr, *d_dec = nullptr;
  const size_t npt = ent_mode ? 1 : (size_t)batch * cap;
  bool ok = hipMalloc(&d_g, (2 * n + 9 + 4) * 8) == hipSuccess && hipMalloc(&d_mu, (size_t)batch * 4 * 8) == hipSuccess &&
            hipMalloc(&d_px, npt * 8) == hipSuccess && hipMalloc(&d_py, npt * 8) == hipSuccess &&
            hipMalloc(&d_pw, npt * 8) == hipSuccess && hipMalloc(&d_out, (size_t)batch * nout * 8) == hipSuccess &&
            hipMalloc(&d_np, batch * 4) == hipSuccess && hipMalloc(&d_err, batch * 4) == hipSuccess &&
            (!ent_mode || hipMalloc(&d_dec, (size_t)n_entries * 8 * 4 * (entries_per_rule ? batch : 1)) == hipSuccess);
  auto release = [&]() {
    for (void* ptr : {(void*)d_g, (void*)d_mu, (void*)d_px, (void*)d_py, (void*)d_pw, (void*)d_out, (void*)d_np,
                      (void*)d_err, (void*)d_dec})
      if (ptr) hipFree(ptr);
  };
  if (!ok) {
    release();
    return off_fail(c, LBDDC_E_NOMEM, "implicit_tensors: device allocation failed");
  }
  std::vector<double> tab(gx);
  tab.insert(tab.end(), gw.begin(), gw.end());
  tab.insert(tab.end(), nodes.begin(), nodes.end());
  tab.insert(tab.end(), qnodes.begin(), qnodes.end());
  hipError_t e = hipMemcpy(d_g, tab.data(), tab.size() * 8, hipMemcpyHostToDevice);
  // entry e of a rule decoded as {a1, b1, j1, a2, b2, j2, a3, b3}
  auto decode = [&](const int64_t* ent, size_t n, std::vector<int>& dec) {
    dec.resize(n * 8);
    const int P1 = p + 1, Q1 = q + 1;
    for (size_t k = 0; k < n; ++k) {
      long long idx = ent[k];
      const int k3 = (int)(idx % nL);
      idx /= nL;
      const int j2 = (int)(idx & 1), j1 = (int)((idx >> 1) & 1);
      idx >>= 2;
      const int k2 = (int)(idx % nB), k1 = (int)(idx / nB);
      const int v[8] = {k1 % P1, k1 / P1, j1, k2 % P1, k2 / P1, j2, k3 % Q1, k3 / Q1};
      for (int j = 0; j < 8; ++j) dec[k * 8 + j] = v[j];
    }
  };
  std::vector<int> dec;
  if (e == hipSuccess && ent_mode && !entries_per_rule) {
    decode(entries, (size_t)n_entries, dec);
    e = hipMemcpy(d_dec, dec.data(), dec.size() * 4, hipMemcpyHostToDevice);
  }
  rule::Cfg cfg{n, d_g, d_g + n, 24};
  SnapArgs sa{d_px, d_py, d_pw, d_np, cap, p, q, nB, nL, d_g + 2 * n, d_g + 2 * n + (p + 1), d_out, n_i};
  std::vector<int> err(batch);
  for (int b0 = 0; b0 < count && e == hipSuccess; b0 += batch) {
    const int nb = std::min(batch, count - b0);
    e = hipMemcpyAsync(d_mu, mu + (size_t)b0 * 4, (size_t)nb * 4 * 8, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) break;
    if (ent_mode && entries_per_rule) {
      decode(entries + (size_t)b0 * n_entries, (size_t)nb * n_entries, dec);
      e = hipMemcpy(d_dec, dec.data(), dec.size() * 4, hipMemcpyHostToDevice);
      if (e != hipSuccess) break;
    }
    if (ent_mode)
      hipLaunchKernelGGL(k_rule_entries, dim3((nb + 63) / 64), dim3(64), 0, c->stream, d_mu, (int)family, nb, cfg, p, q,
                         sa.nodes, sa.qnodes, d_dec, (int)n_entries, entries_per_rule ? 8 * (int)n_entries : 0, d_out,
                         d_err);
    else
      hipLaunchKernelGGL(k_rules, dim3((nb + 63) / 64), dim3(64), 0, c->stream, d_mu, (int)family, nb, cfg, d_px, d_py,
                         d_pw, cap, d_np, d_err);
    e = hipMemcpyAsync(err.data(), d_err, nb * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) break;
    for (int i = 0; i < nb; ++i)
      if (err[i]) {
        release();
        return off_fail(c, LBDDC_E_NUMERIC,
                        err[i] == 1 ? "implicit_tensors: a rule needs more than 131072 points"
                                    : "implicit_tensors: quadrature of a trimmed cell failed (root or stack limit)");
      }
    if (!ent_mode) hipLaunchKernelGGL(k_snap_tensor, dim3(nB, nb), dim3(128), 0, c->stream, sa);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(out + (size_t)b0 * nout, d_out, (size_t)nb * nout * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  release();
  if (e != hipSuccess) return off_fail(c, LBDDC_E_HIP, std::string("implicit_tensors: ") + hipGetErrorString(e));
  return LBDDC_OK;
}

extern "C" lbddc_status lbddc_implicit_rule_host(int32_t family, const double* mu, int32_t n, int32_t cap, double* x,
                                                 double* y, double* w, int32_t* count) {
  if (family < 2 || family > 5 || !mu || !x || !y || !w || !count || n < 1 || n > rule::kMaxN || cap < 1)
    return LBDDC_E_ARG;
  std::vector<double> gx, gw;
  gauss_rule(n, gx, gw);
  rule::Cell cl;
  cl.fam = family;
  for (int k = 0; k < 4; ++k) cl.mu[k] = mu[k];
  rule::Cfg cfg{n, gx.data(), gw.data(), 24};
  rule::Out o{x, y, w, cap, 0, 0};
  rule::cell_rule(cl, cfg, o);
  *count = o.n;
  if (o.err) return LBDDC_E_NUMERIC;
  return LBDDC_OK;
}
