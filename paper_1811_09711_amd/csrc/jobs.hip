// Creation of one integration job's device state, shared by the single
// integrator and the batched / serving engines, plus the host-side error
// state and the combination of iterations.
//
// Brass, Kilian, Reuter, arXiv:1811.09711: Sec. 3.2 (grids start
// equidistant), Sec. 3.4 (alpha starts at 1/K), Sec. 3.5 (iterations are
// combined into the final estimate with their variances).
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "mcv_host.h"

namespace mcv {

namespace {

thread_local std::string g_err;

// The installed allocator, and which allocator made each live block.
struct Allocator {
  mcv_alloc_fn alloc = nullptr;
  mcv_free_fn release = nullptr;
  void* ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;
std::unordered_map<void*, Allocator> g_blocks;

// Sub-allocation of one block: every array starts on a 256-byte boundary.
// With base == nullptr it only measures.
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  void take(T*& p, size_t count) {
    off = (off + 255) & ~(size_t)255;
    p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (count > 0 ? count : 1) * sizeof(T);
  }
};

// The arrays uploaded from the host, in block order (the staged prefix).
void carve_inputs(JobDev& j, Carve& c) {
  const size_t d = j.d, K = j.K, P = j.P;
  c.take(j.ckind, K * d);
  c.take(j.cloc, K * d);
  c.take(j.cwidth, K * d);
  c.take(j.pkind, P * d);
  c.take(j.ploc, P * d);
  c.take(j.pwidth, P * d);
  c.take(j.pweight, P);
  c.take(j.twin_peak, K);
  c.take(j.orphans, P);
  c.take(j.iter_dev, 1);
}

void carve_state(JobDev& j, Carve& c) {
  const size_t d = j.d, K = j.K, n = j.n, P = j.P, tsz = j.prec == 1 ? 4 : 8;
  c.take(j.self, 1);
  c.take(j.cmap64, K * d);
  c.take(j.cmap32, K * d);
  c.take(j.cnorm64, K);
  c.take(j.cnorm32, K);
  c.take(j.pmap64, P * d);
  c.take(j.pmap32, P * d);
  c.take(j.pnorm64, P);
  c.take(j.pnorm32, P);
  c.take(j.ctype, K);
  c.take(j.twin_pn64, K);
  c.take(j.twin_pn32, K);
  c.take(j.edges, K * d * (n + 1));
  char* xt = nullptr;
  char* pt = nullptr;
  c.take(xt, K * d * (size_t)j.sT * 2 * tsz);
  c.take(pt, K * d * (size_t)j.sT * 2 * tsz);
  j.xtab = xt;
  j.ptab = pt;
  char* ct = nullptr;
  c.take(ct, K * d * (size_t)j.M * 4 * tsz);
  j.ctab = ct;
  char* gb = nullptr;
  c.take(gb, K * tsz);
  j.gbound = gb;
  char* at = nullptr;
  c.take(at, 3 * K * tsz);
  j.aterm = at;
  char* tat = nullptr;
  c.take(tat, 3 * K * tsz);
  j.t_aterm = tat;
  char* ga = nullptr;
  c.take(ga, K * d * 2 * tsz);
  j.gab = ga;
  c.take(j.hab, K * d * 2);
  c.take(j.skx, K * 2);
  c.take(j.alpha, K);
  c.take(j.nc, K);
  c.take(j.start, K + 1);
  c.take(j.t_alpha, K);
  c.take(j.t_nc, K);
  c.take(j.t_start, K + 1);
  c.take(j.nr, K);
  c.take(j.spb, K);
  c.take(j.bstart, K + 1);
  c.take(j.t_nr, K);
  c.take(j.t_spb, K);
  c.take(j.hist, K * d * n);
  c.take(j.chstats, K * kStatStride);
  c.take(j.history, (size_t)j.max_iter * kHistStride);
  c.take(j.mrg, j.rng ? (size_t)kMrgTables * kMrgEntry + (K + 1) * 6 : 0);
}

// MRG32k3a jump tables and stream starts (layout: JobDev::mrg), from the
// generator's matrices by repeated squaring.
struct Mat3x2 {
  uint32_t a[9], b[9];
};

Mat3x2 mrg_mul(const Mat3x2& x, const Mat3x2& y) {
  Mat3x2 r;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      uint64_t sa = 0, sb = 0;
      for (int q = 0; q < 3; ++q) {
        sa += mrg_mod1((uint64_t)x.a[3 * i + q] * y.a[3 * q + k]);
        sb += mrg_mod2((uint64_t)x.b[3 * i + q] * y.b[3 * q + k]);
      }
      r.a[3 * i + k] = mrg_mod1(sa);
      r.b[3 * i + k] = mrg_mod2(sb);
    }
  return r;
}

void mrg_vec(const Mat3x2& m, uint32_t s[6]) {
  uint32_t r[6];
  for (int i = 0; i < 3; ++i) {
    uint64_t sa = 0, sb = 0;
    for (int q = 0; q < 3; ++q) {
      sa += mrg_mod1((uint64_t)m.a[3 * i + q] * s[q]);
      sb += mrg_mod2((uint64_t)m.b[3 * i + q] * s[3 + q]);
    }
    r[i] = mrg_mod1(sa);
    r[3 + i] = mrg_mod2(sb);
  }
  for (int i = 0; i < 6; ++i) s[i] = r[i];
}

std::vector<uint32_t> mrg_host_tables(uint64_t seed, int K) {
  std::vector<Mat3x2> pw(191);  // pw[b] = A^(2^b)
  pw[0] = Mat3x2{{0, 1, 0, 0, 0, 1, kMrgM1 - 810728u, 1403580u, 0},
                 {0, 1, 0, 0, 0, 1, kMrgM2 - 1370589u, 0, 527612u}};
  for (int b = 1; b < 191; ++b) pw[b] = mrg_mul(pw[b - 1], pw[b - 1]);
  std::vector<uint32_t> out((size_t)kMrgTables * kMrgEntry + (size_t)(K + 1) * 6);
  for (int b = 0; b < 64; ++b) {
    memcpy(&out[(size_t)b * kMrgEntry], &pw[b], sizeof(Mat3x2));
    memcpy(&out[(size_t)(kMrgSubBase + b) * kMrgEntry], &pw[76 + b], sizeof(Mat3x2));
  }
  for (int c = 0; c <= K; ++c) {
    uint64_t g = 1024 * seed + (uint64_t)(c < K ? c : 1023);
    uint32_t st[6] = {12345, 12345, 12345, 12345, 12345, 12345};
    for (int b = 0; g != 0; ++b, g >>= 1)
      if (g & 1) mrg_vec(pw[127 + b], st);
    memcpy(&out[(size_t)kMrgTables * kMrgEntry + (size_t)c * 6], st, sizeof st);
  }
  return out;
}

}  // namespace

mcv_status fail(mcv_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

const char* last_error() { return g_err.c_str(); }

mcv_status set_allocator(mcv_alloc_fn alloc, mcv_free_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(MCV_E_INVALID, "give both allocator functions, or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = Allocator{alloc, release, ctx};
  return MCV_OK;
}

hipError_t dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  Allocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
  }
  if (!a.alloc) {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_alloc_mu);
      g_blocks[*p] = a;
    }
    return e;
  }
  void* q = a.alloc(bytes, a.ctx);
  if (!q) return hipErrorOutOfMemory;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_blocks[q] = a;
  *p = q;
  return hipSuccess;
}

void dev_free(void* p) {
  if (!p) return;
  Allocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_blocks.find(p);
    if (it == g_blocks.end()) return;  // not ours
    a = it->second;
    g_blocks.erase(it);
  }
  if (!a.release) {
    (void)hipFree(p);
    return;
  }
  (void)hipDeviceSynchronize();
  a.release(p, a.ctx);
}

mcv_status validate_problem(const mcv_problem* p) {
  if (!p) return fail(MCV_E_INVALID, "problem is NULL");
  if (p->dim < 1 || p->dim > 32) return fail(MCV_E_INVALID, "dim must be in [1, 32]");
  if (p->n_bins < 1 || p->n_bins > 256) return fail(MCV_E_INVALID, "n_bins must be in [1, 256]");
  if (p->n_channels < 1 || p->n_channels > 1024)
    return fail(MCV_E_INVALID, "n_channels must be in [1, 1024]");
  if (p->n_peaks < 1 || p->n_peaks > 1024) return fail(MCV_E_INVALID, "n_peaks must be in [1, 1024]");
  if (p->precision != MCV_FP64 && p->precision != MCV_FP32_MIXED)
    return fail(MCV_E_INVALID, "precision must be MCV_FP64 or MCV_FP32_MIXED");
  if (!p->peak_kind || !p->peak_loc || !p->peak_width || !p->peak_weight || !p->chan_kind ||
      !p->chan_loc || !p->chan_width)
    return fail(MCV_E_INVALID, "a problem array is NULL");
  if (!(p->grid_power >= 0.0) || !isfinite(p->grid_power))
    return fail(MCV_E_INVALID, "grid_power must be finite and >= 0");
  if (!(p->channel_power >= 0.0) || !isfinite(p->channel_power))
    return fail(MCV_E_INVALID, "channel_power must be finite and >= 0");
  if (p->min_calls < 1) return fail(MCV_E_INVALID, "min_calls must be >= 1");
  if (p->strat < 0 || p->strat == 1 || p->strat > (1 << 20))
    return fail(MCV_E_INVALID, "strat must be 0 (uniform) or the calls per box, 2..2^20");
  if (p->rng != MCV_RNG_PHILOX && p->rng != MCV_RNG_MRG32K3A)
    return fail(MCV_E_INVALID, "rng must be MCV_RNG_PHILOX or MCV_RNG_MRG32K3A");
  if (p->rng == MCV_RNG_MRG32K3A && (p->n_channels > 1023 || p->seed >= ((uint64_t)1 << 54)))
    return fail(MCV_E_INVALID, "MRG32k3a streams need n_channels <= 1023 and seed < 2^54");
  if (p->max_iterations < 1) return fail(MCV_E_INVALID, "max_iterations must be >= 1");
  auto check = [&](const int32_t* kind, const double* loc, const double* width, int n,
                   const char* what) -> mcv_status {
    for (int i = 0; i < n * p->dim; ++i) {
      if (kind[i] != MCV_FLAT && kind[i] != MCV_GAUSS && kind[i] != MCV_BW)
        return fail(MCV_E_INVALID, std::string(what) + ": unknown kind");
      if (kind[i] == MCV_FLAT) continue;
      if (!(width[i] > 0.0) || !isfinite(width[i]))
        return fail(MCV_E_INVALID, std::string(what) + ": width must be finite and > 0");
      if (!(loc[i] >= 0.0 && loc[i] <= 1.0))
        return fail(MCV_E_INVALID, std::string(what) + ": centre must lie in [0, 1]");
    }
    return MCV_OK;
  };
  mcv_status st = check(p->peak_kind, p->peak_loc, p->peak_width, p->n_peaks, "peak");
  if (st != MCV_OK) return st;
  st = check(p->chan_kind, p->chan_loc, p->chan_width, p->n_channels, "channel");
  if (st != MCV_OK) return st;
  for (int i = 0; i < p->n_peaks; ++i)
    if (!isfinite(p->peak_weight[i])) return fail(MCV_E_INVALID, "peak weight must be finite");
  return MCV_OK;
}

mcv_status device_cus(int* device, int* n_cu) {
  hipError_t e = hipGetDevice(device);
  int ncu = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, *device);
  if (e != hipSuccess) return fail(MCV_E_DEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  *n_cu = ncu > 0 ? ncu : 1;
  return MCV_OK;
}

size_t partial_bytes(const JobDev& j, int G) {
  const size_t slots = (size_t)G + (size_t)j.K;
  const size_t a = (slots * kPartStride * sizeof(double) + 255) & ~(size_t)255;
  return a + slots * (size_t)j.d * j.n * sizeof(double);
}

void carve_partials(JobDev& j, int G, char* base) {
  const size_t slots = (size_t)G + (size_t)j.K;
  const size_t a = (slots * kPartStride * sizeof(double) + 255) & ~(size_t)255;
  j.part = reinterpret_cast<double*>(base);
  j.hpart = reinterpret_cast<double*>(base + a);
  j.gmax = G;
}

size_t job_block_bytes(const mcv_problem* p, int gmax) {
  JobDev j;
  j.d = p->dim;
  j.K = p->n_channels;
  j.n = p->n_bins;
  j.P = p->n_peaks;
  j.prec = p->precision;
  j.sT = (j.n + 3) & ~1;
  j.M = hint_cells_for_bins(j.n);
  j.mshift = hint_cell_shift(j.M);
  j.max_iter = p->max_iterations;
  j.rng = p->rng;
  j.strat = p->strat;
  Carve m;
  carve_inputs(j, m);
  carve_state(j, m);
  size_t total = m.off;
  if (gmax > 0) total = ((total + 255) & ~(size_t)255) + partial_bytes(j, gmax);
  return total;
}

mcv_status job_create(const mcv_problem* p, int gmax, int64_t n_points, int n_cu, hipStream_t s,
                      JobDev* out, void** block) {
  *block = nullptr;
  mcv_status st = validate_problem(p);
  if (st != MCV_OK) return st;
  JobDev j;
  j.d = p->dim;
  j.K = p->n_channels;
  j.n = p->n_bins;
  j.P = p->n_peaks;
  j.prec = p->precision;
  j.npow2 = 1;
  while (j.npow2 < j.n) j.npow2 <<= 1;
  j.sT = (j.n + 3) & ~1;  // entries 0..n+1, even
  j.M = hint_cells_for_bins(j.n);
  j.mshift = hint_cell_shift(j.M);
  j.n_cu = n_cu;
  j.seed = p->seed;
  j.grid_power = p->grid_power;
  j.channel_power = p->channel_power;
  j.min_calls = p->min_calls;
  j.max_iter = p->max_iterations;
  j.n_points = n_points;
  j.rng = p->rng;
  j.strat = p->strat;
  if (sample_lds_bytes(j) > 160 * 1024)
    return fail(MCV_E_INVALID, "dim * n_bins too large for the LDS of one workgroup");
  const size_t d = j.d, K = j.K, P = j.P;

  // channels whose map has the exact shape of a peak share that peak's
  // exponential; each peak is claimed by at most one channel
  std::vector<int32_t> twin(K, -1), orphan;
  {
    std::vector<char> taken(P, 0);
    for (size_t c = 0; c < K; ++c)
      for (size_t i = 0; i < P && twin[c] < 0; ++i) {
        if (taken[i]) continue;
        bool same = true;
        for (size_t k = 0; k < d && same; ++k) {
          const size_t a = c * d + k, b = i * d + k;
          if (p->chan_kind[a] != p->peak_kind[b]) same = false;
          else if (p->chan_kind[a] != MCV_FLAT &&
                   (p->chan_loc[a] != p->peak_loc[b] || p->chan_width[a] != p->peak_width[b]))
            same = false;
        }
        if (same) {
          twin[c] = (int32_t)i;
          taken[i] = 1;
        }
      }
    for (size_t i = 0; i < P; ++i)
      if (!taken[i]) orphan.push_back((int32_t)i);
  }
  j.n_orphan = (int)orphan.size();

  // measure, allocate, carve
  Carve m;
  carve_inputs(j, m);
  const size_t staged = m.off;
  carve_state(j, m);
  size_t total = m.off;
  size_t part_off = 0;
  if (gmax > 0) {
    part_off = (total + 255) & ~(size_t)255;
    total = part_off + partial_bytes(j, gmax);
  }
  void* dev = nullptr;
  hipError_t e = dev_alloc(&dev, total);
  if (e != hipSuccess) return fail(MCV_E_NOMEM, std::string("job block: ") + hipGetErrorString(e));
  Carve c;
  c.base = static_cast<char*>(dev);
  carve_inputs(j, c);
  carve_state(j, c);
  if (gmax > 0) carve_partials(j, gmax, static_cast<char*>(dev) + part_off);

  // stage the inputs in the block's own layout: one upload
  std::vector<char> stage(staged, 0);
  JobDev h = j;
  Carve hc;
  hc.base = stage.data();
  carve_inputs(h, hc);
  memcpy(h.ckind, p->chan_kind, K * d * sizeof(int32_t));
  memcpy(h.cloc, p->chan_loc, K * d * sizeof(double));
  memcpy(h.cwidth, p->chan_width, K * d * sizeof(double));
  memcpy(h.pkind, p->peak_kind, P * d * sizeof(int32_t));
  memcpy(h.ploc, p->peak_loc, P * d * sizeof(double));
  memcpy(h.pwidth, p->peak_width, P * d * sizeof(double));
  memcpy(h.pweight, p->peak_weight, P * sizeof(double));
  memcpy(h.twin_peak, twin.data(), K * sizeof(int32_t));
  if (!orphan.empty()) memcpy(h.orphans, orphan.data(), orphan.size() * sizeof(int32_t));
  *h.iter_dev = 0;

  e = hipMemcpyAsync(dev, stage.data(), staged, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(j.self, &j, sizeof(JobDev), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemsetAsync(j.history, 0, (size_t)j.max_iter * kHistStride * sizeof(double), s);
  std::vector<uint32_t> mrg_tab;
  if (e == hipSuccess && j.rng) {
    mrg_tab = mrg_host_tables(j.seed, j.K);
    e = hipMemcpyAsync(j.mrg, mrg_tab.data(), mrg_tab.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) {
    launch_setup(j, s);
    launch_tables(single_set(j), s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // stage and j are read until here
  if (e != hipSuccess) {
    dev_free(dev);
    return fail(MCV_E_DEVICE, std::string("job set-up: ") + hipGetErrorString(e));
  }
  *out = j;
  *block = dev;
  return MCV_OK;
}

void combine_history(const double* hist, int n, int first, mcv_summary* out) {
  double sw = 0.0, swe = 0.0, zsum = 0.0, npts = 0.0, nbad = 0.0;
  int nz = 0, used = 0;
  for (int t = first; t < n; ++t) {
    const double* r = &hist[(size_t)t * kHistStride];
    ++used;
    npts += r[2];
    nbad += r[4];
    if (r[1] == 0.0) {
      zsum += r[0];
      ++nz;
    } else {
      sw += 1.0 / (r[1] * r[1]);
      swe += r[0] / (r[1] * r[1]);
    }
  }
  memset(out, 0, sizeof *out);
  out->n_iter_used = used;
  out->n_points = (int64_t)npts;
  out->n_bad = (int64_t)nbad;
  out->w_max = hist[(size_t)(n - 1) * kHistStride + 3];
  if (nz > 0) {
    out->integral = zsum / nz;
    return;
  }
  const double mean = swe / sw;
  double chi2 = 0.0;
  for (int t = first; t < n; ++t) {
    const double* r = &hist[(size_t)t * kHistStride];
    chi2 += (r[0] - mean) * (r[0] - mean) / (r[1] * r[1]);
  }
  out->integral = mean;
  out->error = 1.0 / sqrt(sw);
  out->chi2_ndf = used > 1 ? chi2 / (used - 1) : 0.0;
}

}  // namespace mcv
