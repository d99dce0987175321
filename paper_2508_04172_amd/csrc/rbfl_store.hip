// Saving and loading a built handle: the start-up stage's artefacts (frame,
// nodes, RBF weights, SVD basis and its spline-folded copy, node series,
// output layout, the online stage's constants and the exact likelihood's band
// data), so that the sampling stage can reuse a start-up without repeating it
// (Sec. II D: the interpolants are built once and then only evaluated).
//
// File layout (host byte order): the 8-byte magic, a u32 format version, the
// u32 ABI version, a u64 section count, then sections {u32 tag, u32 element
// bytes, u64 element count, payload}, then a u64 checksum of everything
// before it (FNV-1a over 8-byte words, the tail zero-padded).  Loading checks
// the magic, both versions, the checksum, that every section is present once
// with the element size and count the sizes section implies, and that the
// constants agree with those sizes; any failure is RBFL_E_INVALID_ARG and
// allocates nothing on the device.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "rbfl_internal.h"

namespace rbfl {

namespace {

constexpr char kMagic[8] = {'R', 'B', 'F', 'L', 'S', 'T', 'O', 'R'};
constexpr uint32_t kFormat = 1;

enum Tag : uint32_t {
  kScalars = 1,
  kConsts,
  kXNodes,
  kPhysNodes,
  kNodeValues,
  kSingular,
  kNodesDev,
  kWeights,
  kBasis,
  kBasis4,
  kZNodes,
  kBruteD,
  kBruteW,
  kColdesc,
  kBands,
  kTagEnd
};

// Every scalar of a built handle that the online stage, the exact likelihood
// and the queries read.
struct Scalars {
  int32_t n_det, n_modes, modes[RBFL_MAX_MODES][2];
  int32_t N, M, K, Kp, rows, q, T, half_w, degree;
  int32_t n_bands, n_v;
  int64_t n_s, n_f, brute_j_lo, brute_J;
  double fs, seg_len, f_low, df, eps, chi_max, t_trig, d_ref, match, f_ref, earth_rate;
  double squeeze[2], centre_opt[6], centre_snr[2];
  double theta_c[4], V[16], lam[4], semi[4], metric[16];
  double D[RBFL_MAX_DET][9], r[RBFL_MAX_DET][3];
  double cond, timing[8];
};

uint64_t fnv_words(uint64_t h, const unsigned char *p, size_t n) {
  const uint64_t prime = 0x100000001b3ull;
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    std::memcpy(&w, p + i, 8);
    h = (h ^ w) * prime;
  }
  if (i < n) {
    uint64_t w = 0;
    std::memcpy(&w, p + i, n - i);
    h = (h ^ w) * prime;
  }
  return h;
}

struct Section {
  uint32_t tag, esize;
  uint64_t count;
  std::vector<unsigned char> data;
};

template <class T>
Section host_section(uint32_t tag, const T *p, size_t count) {
  Section s{tag, (uint32_t)sizeof(T), count, {}};
  s.data.resize(sizeof(T) * count);
  if (count) std::memcpy(s.data.data(), p, s.data.size());
  return s;
}

template <class T>
Section device_section(uint32_t tag, const DevBuf<T> &b) {
  Section s{tag, (uint32_t)sizeof(T), b.n, {}};
  s.data.resize(sizeof(T) * b.n);
  if (b.n) RBFL_HIP(hipMemcpy(s.data.data(), b.p, s.data.size(), hipMemcpyDeviceToHost));
  return s;
}

struct File {
  FILE *f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

void save(const Ctx &c, const char *path) {
  require(path != nullptr, "path is NULL");
  Scalars sc;
  std::memset(&sc, 0, sizeof(sc));
  sc.n_det = c.n_det;
  sc.n_modes = c.n_modes;
  std::memcpy(sc.modes, c.modes, sizeof(sc.modes));
  sc.N = c.N;
  sc.M = c.M;
  sc.K = c.K;
  sc.Kp = c.Kp;
  sc.rows = c.rows;
  sc.q = c.q;
  sc.T = c.T;
  sc.half_w = c.half_w;
  sc.degree = c.degree;
  sc.n_bands = c.n_bands;
  sc.n_v = c.n_v;
  sc.n_s = c.n_s;
  sc.n_f = c.n_f;
  sc.brute_j_lo = c.brute_j_lo;
  sc.brute_J = c.brute_J;
  sc.fs = c.fs;
  sc.seg_len = c.seg_len;
  sc.f_low = c.f_low;
  sc.df = c.df;
  sc.eps = c.eps;
  sc.chi_max = c.chi_max;
  sc.t_trig = c.t_trig;
  sc.d_ref = c.d_ref;
  sc.match = c.match;
  sc.f_ref = c.f_ref;
  sc.earth_rate = c.earth_rate;
  std::memcpy(sc.squeeze, c.squeeze, sizeof(sc.squeeze));
  std::memcpy(sc.centre_opt, c.centre_opt, sizeof(sc.centre_opt));
  std::memcpy(sc.centre_snr, c.centre_snr, sizeof(sc.centre_snr));
  std::memcpy(sc.theta_c, c.theta_c, sizeof(sc.theta_c));
  std::memcpy(sc.V, c.V, sizeof(sc.V));
  std::memcpy(sc.lam, c.lam, sizeof(sc.lam));
  std::memcpy(sc.semi, c.semi, sizeof(sc.semi));
  std::memcpy(sc.metric, c.metric, sizeof(sc.metric));
  std::memcpy(sc.D, c.D, sizeof(sc.D));
  std::memcpy(sc.r, c.r, sizeof(sc.r));
  sc.cond = c.cond;
  std::memcpy(sc.timing, c.timing, sizeof(sc.timing));

  RBFL_HIP(hipDeviceSynchronize());
  std::vector<Section> secs;
  secs.push_back(host_section(kScalars, &sc, 1));
  secs.push_back(host_section(kConsts, &c.host_consts, 1));
  secs.push_back(host_section(kXNodes, c.x_nodes.data(), c.x_nodes.size()));
  secs.push_back(host_section(kPhysNodes, c.phys_nodes.data(), c.phys_nodes.size()));
  secs.push_back(host_section(kNodeValues, c.node_values.data(), c.node_values.size()));
  secs.push_back(host_section(kSingular, c.singular.data(), c.singular.size()));
  secs.push_back(device_section(kNodesDev, c.nodes));
  secs.push_back(device_section(kWeights, c.W));
  secs.push_back(device_section(kBasis, c.basis));
  secs.push_back(device_section(kBasis4, c.basis4));
  secs.push_back(device_section(kZNodes, c.z_nodes));
  secs.push_back(device_section(kBruteD, c.brute_D));
  secs.push_back(device_section(kBruteW, c.brute_w));
  secs.push_back(device_section(kColdesc, c.coldesc));
  secs.push_back(host_section(kBands, c.band_edges.data(), c.band_edges.size()));

  // written to a temporary name and renamed, so that a failed save leaves no
  // partial file under `path`
  const std::string tmp = std::string(path) + ".tmp";
  {
    File out;
    out.f = std::fopen(tmp.c_str(), "wb");
    if (!out.f) throw Error(RBFL_E_INVALID_ARG, std::string("cannot open ") + tmp + " for writing");
    uint64_t h = 0xcbf29ce484222325ull;
    bool ok = true;
    auto put = [&](const void *p, size_t n) {
      if (!ok || n == 0) return;
      ok = std::fwrite(p, 1, n, out.f) == n;
    };
    // the checksum runs over 8-byte words of a stream built from 8-byte-aligned
    // pieces: header (24 bytes), each section header (16) and payload padded to 8
    std::vector<unsigned char> head(24, 0);
    std::memcpy(head.data(), kMagic, 8);
    std::memcpy(head.data() + 8, &kFormat, 4);
    const uint32_t abi = RBFL_ABI_VERSION;
    std::memcpy(head.data() + 12, &abi, 4);
    const uint64_t ns = secs.size();
    std::memcpy(head.data() + 16, &ns, 8);
    put(head.data(), head.size());
    h = fnv_words(h, head.data(), head.size());
    for (const Section &s : secs) {
      unsigned char sh[16];
      std::memcpy(sh, &s.tag, 4);
      std::memcpy(sh + 4, &s.esize, 4);
      std::memcpy(sh + 8, &s.count, 8);
      put(sh, 16);
      h = fnv_words(h, sh, 16);
      put(s.data.data(), s.data.size());
      h = fnv_words(h, s.data.data(), s.data.size());
      const size_t pad = (8 - s.data.size() % 8) % 8;
      const unsigned char zeros[8] = {};
      put(zeros, pad);
    }
    put(&h, 8);
    if (!ok || std::fflush(out.f) != 0) {
      std::remove(tmp.c_str());
      throw Error(RBFL_E_INVALID_ARG, std::string("write to ") + tmp + " failed");
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    throw Error(RBFL_E_INVALID_ARG, std::string("cannot rename ") + tmp + " to " + path);
  }
}

void corrupt(const std::string &why) { throw Error(RBFL_E_INVALID_ARG, "not a valid rbfl store file: " + why); }

std::vector<unsigned char> read_all(const char *path) {
  File in;
  in.f = std::fopen(path, "rb");
  if (!in.f) throw Error(RBFL_E_INVALID_ARG, std::string("cannot open ") + path);
  std::vector<unsigned char> buf;
  unsigned char tmp[1 << 16];
  size_t n;
  while ((n = std::fread(tmp, 1, sizeof(tmp), in.f)) > 0) buf.insert(buf.end(), tmp, tmp + n);
  if (std::ferror(in.f)) throw Error(RBFL_E_INVALID_ARG, std::string("read of ") + path + " failed");
  return buf;
}

template <class T>
void upload(DevBuf<T> &b, const Section &s, hipStream_t st) {
  b.alloc(s.count);
  if (s.count) RBFL_HIP(hipMemcpyAsync(b.p, s.data.data(), s.data.size(), hipMemcpyHostToDevice, st));
}

template <class T>
void to_vector(std::vector<T> &v, const Section &s) {
  v.resize(s.count);
  if (s.count) std::memcpy(v.data(), s.data.data(), s.data.size());
}

void load(const char *path, hipStream_t st, Ctx &c) {
  require(path != nullptr, "path is NULL");
  const std::vector<unsigned char> buf = read_all(path);
  // checksum first: nothing of a damaged file is interpreted
  if (buf.size() < 32 || buf.size() % 8 != 0) corrupt("truncated");
  const size_t body = buf.size() - 8;
  uint64_t stored;
  std::memcpy(&stored, buf.data() + body, 8);
  if (fnv_words(0xcbf29ce484222325ull, buf.data(), body) != stored) corrupt("checksum mismatch");
  if (std::memcmp(buf.data(), kMagic, 8) != 0) corrupt("bad magic");
  uint32_t fmt, abi;
  uint64_t ns;
  std::memcpy(&fmt, buf.data() + 8, 4);
  std::memcpy(&abi, buf.data() + 12, 4);
  std::memcpy(&ns, buf.data() + 16, 8);
  if (fmt != kFormat) corrupt("format version " + std::to_string(fmt) + " (this library reads " + std::to_string(kFormat) + ")");
  if (abi != RBFL_ABI_VERSION) corrupt("written by ABI version " + std::to_string(abi));
  if (ns != kTagEnd - 1) corrupt("section count");
  std::vector<Section> secs(kTagEnd);
  std::vector<bool> seen(kTagEnd, false);
  size_t off = 24;
  for (uint64_t i = 0; i < ns; ++i) {
    if (off + 16 > body) corrupt("truncated section header");
    Section s;
    std::memcpy(&s.tag, buf.data() + off, 4);
    std::memcpy(&s.esize, buf.data() + off + 4, 4);
    std::memcpy(&s.count, buf.data() + off + 8, 8);
    off += 16;
    if (s.tag == 0 || s.tag >= kTagEnd || seen[s.tag]) corrupt("section tag");
    if (s.esize == 0 || s.count > (body - off) / s.esize) corrupt("section size");
    const size_t bytes = (size_t)s.esize * s.count;
    s.data.assign(buf.data() + off, buf.data() + off + bytes);
    off += bytes + (8 - bytes % 8) % 8;
    if (off > body) corrupt("truncated section");
    seen[s.tag] = true;
    secs[s.tag] = std::move(s);
  }
  if (off != body) corrupt("trailing bytes");
  auto need = [&](uint32_t tag, size_t esize, uint64_t count) -> const Section & {
    const Section &s = secs[tag];
    if (s.esize != esize || s.count != count) corrupt("section " + std::to_string(tag) + " has the wrong size");
    return s;
  };
  Scalars sc;
  std::memcpy(&sc, need(kScalars, sizeof(Scalars), 1).data.data(), sizeof(Scalars));
  // the sizes must be those of a handle this library can build
  if (sc.n_det < 1 || sc.n_det > RBFL_MAX_DET || sc.n_modes < 1 || sc.n_modes > RBFL_MAX_MODES) corrupt("sizes");
  if (sc.degree < 0 || sc.degree > 3 || sc.N < 1 || sc.q < 1 || sc.T < 1 || sc.half_w < 0 || sc.T != 2 * sc.half_w + 1)
    corrupt("sizes");
  static const int kMonomials[4] = {1, 5, 15, 35};
  if (sc.M != kMonomials[sc.degree]) corrupt("sizes");
  if (sc.n_bands < 1 || sc.n_bands > RBFL_MAX_BANDS || sc.n_v != sc.n_det * sc.n_bands || sc.n_v > RBFL_MAX_BLOCKS)
    corrupt("sizes");
  if (sc.K != sc.n_v * (2 * sc.q * sc.n_modes + sc.n_modes * sc.n_modes)) corrupt("sizes");
  if (sc.Kp != ((sc.K + kColTile - 1) / kColTile) * kColTile) corrupt("sizes");
  if (sc.rows != ((sc.N + sc.M + kRowChunk - 1) / kRowChunk) * kRowChunk) corrupt("sizes");
  if (sc.n_s < 16 || sc.n_f != sc.n_s / 2 + 1 || sc.brute_J < 0 || sc.brute_j_lo < 1 ||
      sc.brute_j_lo + sc.brute_J > sc.n_s / 2 + 1)
    corrupt("sizes");
  const int mn = sc.N < sc.T ? sc.N : sc.T;
  const size_t pairs = (size_t)sc.n_v * sc.n_modes;
  EvalConsts ec;
  std::memcpy(&ec, need(kConsts, sizeof(EvalConsts), 1).data.data(), sizeof(EvalConsts));
  if (ec.n_det != sc.n_det || ec.n_modes != sc.n_modes || ec.N != sc.N || ec.M != sc.M || ec.K != sc.K ||
      ec.Kp != sc.Kp || ec.rows != sc.rows || ec.q != sc.q || ec.T != sc.T || ec.half_w != sc.half_w ||
      ec.degree != sc.degree || ec.n_bands != sc.n_bands || ec.n_v != sc.n_v)
    corrupt("constants disagree with the sizes");
  for (int k = 0; k < sc.n_v; ++k) {
    if (ec.sig_off[k] < 0 || ec.sig_off[k] + sc.n_modes * sc.n_modes > sc.K) corrupt("output layout");
    for (int a = 0; a < sc.n_modes; ++a)
      if (ec.coef_off[k][a] < 0 || ec.coef_off[k][a] + 2 * sc.q > sc.K) corrupt("output layout");
  }
  const Section &xn = need(kXNodes, sizeof(double), (uint64_t)sc.N * 4);
  const Section &pn = need(kPhysNodes, sizeof(double), (uint64_t)sc.N * 4);
  const Section &nv = need(kNodeValues, sizeof(double), (uint64_t)sc.N * sc.K);
  const Section &sv = need(kSingular, sizeof(double), (uint64_t)pairs * mn);
  const Section &nd = need(kNodesDev, sizeof(double), (uint64_t)sc.rows * 4);
  const Section &w = need(kWeights, sizeof(double), (uint64_t)sc.rows * sc.Kp);
  const Section &b = need(kBasis, sizeof(double2), (uint64_t)pairs * sc.T * sc.q);
  const Section &b4 = need(kBasis4, sizeof(double2), (uint64_t)pairs * sc.T * sc.q * 4);
  const Section &zn = need(kZNodes, sizeof(double2), (uint64_t)pairs * sc.N * sc.T);
  const Section &bd = need(kBruteD, sizeof(double2), (uint64_t)sc.n_det * sc.brute_J);
  const Section &bw = need(kBruteW, sizeof(double), (uint64_t)sc.n_det * sc.brute_J);
  const Section &cd = need(kColdesc, sizeof(int4), (uint64_t)sc.K);
  const Section &be = need(kBands, sizeof(int64_t), (uint64_t)sc.n_bands + 1);
  std::vector<int64_t> edges;
  to_vector(edges, be);
  if (edges.front() != sc.brute_j_lo || edges.back() != sc.n_s / 2) corrupt("band edges");
  for (int b = 0; b < sc.n_bands; ++b)
    if (edges[b + 1] < edges[b]) corrupt("band edges");

  RBFL_HIP(hipGetDevice(&c.device));
  c.n_det = sc.n_det;
  c.n_modes = sc.n_modes;
  std::memcpy(c.modes, sc.modes, sizeof(c.modes));
  c.N = sc.N;
  c.M = sc.M;
  c.K = sc.K;
  c.Kp = sc.Kp;
  c.rows = sc.rows;
  c.q = sc.q;
  c.T = sc.T;
  c.half_w = sc.half_w;
  c.degree = sc.degree;
  c.n_bands = sc.n_bands;
  c.n_v = sc.n_v;
  c.band_edges = edges;
  c.n_s = sc.n_s;
  c.n_f = sc.n_f;
  c.brute_j_lo = sc.brute_j_lo;
  c.brute_J = sc.brute_J;
  c.fs = sc.fs;
  c.seg_len = sc.seg_len;
  c.f_low = sc.f_low;
  c.df = sc.df;
  c.eps = sc.eps;
  c.chi_max = sc.chi_max;
  c.t_trig = sc.t_trig;
  c.d_ref = sc.d_ref;
  c.match = sc.match;
  c.f_ref = sc.f_ref;
  c.earth_rate = sc.earth_rate;
  std::memcpy(c.squeeze, sc.squeeze, sizeof(c.squeeze));
  std::memcpy(c.centre_opt, sc.centre_opt, sizeof(c.centre_opt));
  std::memcpy(c.centre_snr, sc.centre_snr, sizeof(c.centre_snr));
  std::memcpy(c.theta_c, sc.theta_c, sizeof(c.theta_c));
  std::memcpy(c.V, sc.V, sizeof(c.V));
  std::memcpy(c.lam, sc.lam, sizeof(c.lam));
  std::memcpy(c.semi, sc.semi, sizeof(c.semi));
  std::memcpy(c.metric, sc.metric, sizeof(c.metric));
  std::memcpy(c.D, sc.D, sizeof(c.D));
  std::memcpy(c.r, sc.r, sizeof(c.r));
  c.cond = sc.cond;
  std::memcpy(c.timing, sc.timing, sizeof(c.timing));
  c.host_consts = ec;
  to_vector(c.x_nodes, xn);
  to_vector(c.phys_nodes, pn);
  to_vector(c.node_values, nv);
  to_vector(c.singular, sv);
  c.consts.alloc(1);
  RBFL_HIP(hipMemcpyAsync(c.consts.p, &c.host_consts, sizeof(EvalConsts), hipMemcpyHostToDevice, st));
  upload(c.nodes, nd, st);
  upload(c.W, w, st);
  upload(c.basis, b, st);
  upload(c.basis4, b4, st);
  upload(c.z_nodes, zn, st);
  upload(c.brute_D, bd, st);
  upload(c.brute_w, bw, st);
  upload(c.coldesc, cd, st);
  c.nan_part.alloc(kNanParts);
  launch_count_nan(nullptr, 0, c.nan_part.p, st);
  RBFL_HIP(hipStreamSynchronize(st));
  if (debug_mode()) debug_check_layout(c);
}

}  // namespace

}  // namespace rbfl

extern "C" {

int32_t rbfl_save(rbfl_handle h, const char *path) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::save(h->c, path);
  });
}

int32_t rbfl_load(const char *path, void *stream, rbfl_handle *out) {
  return rbfl::guarded([&] {
    rbfl::require(out != nullptr, "out is NULL");
    *out = nullptr;
    std::unique_ptr<rbfl_ctx> h(new rbfl_ctx());
    rbfl::load(path, reinterpret_cast<hipStream_t>(stream), h->c);
    *out = h.release();
  });
}

}  // extern "C"
