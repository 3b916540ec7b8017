// MGN1 weights parser and device upload of the CoeffNet/MgNet weights
// (architecture of the paper's Sec. 3.2-3.3).
#include <cmath>
#include <cstring>
#include <map>

#include "common.h"
#include "taps.h"

namespace rte {

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return uint16_t(u >> 16);
}

namespace {

enum Kind {
  K_WIN = 1, K_WOUT, K_S, K_A, K_BPRE, K_BPOST, K_BC, K_R, K_PR,
  K_CW, K_CB, K_HAW, K_HAB, K_HIW, K_HIB
};

struct Rec {
  std::vector<uint32_t> dims;
  const float* data;  // unaligned view into the blob: copied with memcpy
  size_t count;
};

uint32_t rd32(const unsigned char* p) {
  return uint32_t(p[0]) | (uint32_t(p[1]) << 8) | (uint32_t(p[2]) << 16) | (uint32_t(p[3]) << 24);
}

std::vector<float> take(const Rec& r) {
  std::vector<float> v(r.count);
  std::memcpy(v.data(), r.data, r.count * 4);
  for (float x : v)
    if (!std::isfinite(x)) fail(RTE_EFORMAT, "MGN1: non-finite weight");
  return v;
}

// Conv weights stored [cout][cin][taps] -> GEMM layout [tap][cout][cin].
ConvW pack_conv3(const std::vector<float>& w, int cout, int cin, int dim) {
  ConvW c;
  c.taps = dim == 3 ? 27 : 9;
  c.cout = cout;
  c.cin = cin;
  c.f32.resize(size_t(c.taps) * cout * cin);
  for (int co = 0; co < cout; ++co)
    for (int ci = 0; ci < cin; ++ci)
      for (int t = 0; t < c.taps; ++t)
        c.f32[(size_t(t) * cout + co) * cin + ci] = w[(size_t(co) * cin + ci) * c.taps + t];
  return c;
}

// Transposed conv weights stored [cin][cout][4^dim] -> [class][tap][cout][cin].
ConvW pack_convT4(const std::vector<float>& w, int cin, int cout, int dim) {
  ConvW c;
  int ncls = 1 << dim, ntap = 1 << dim, ktot = dim == 3 ? 64 : 16;
  c.taps = ncls * ntap;
  c.cout = cout;
  c.cin = cin;
  c.f32.resize(size_t(c.taps) * cout * cin);
  for (int cls = 0; cls < ncls; ++cls)
    for (int t = 0; t < ntap; ++t) {
      int k[3], off[3];
      convT4_tap(dim, cls, t, k, off);
      int kidx = dim == 3 ? (k[2] * 4 + k[1]) * 4 + k[0] : k[1] * 4 + k[0];
      size_t tt = size_t(cls) * ntap + t;
      for (int co = 0; co < cout; ++co)
        for (int ci = 0; ci < cin; ++ci)
          c.f32[(tt * cout + co) * cin + ci] = w[(size_t(ci) * cout + co) * ktot + kidx];
    }
  return c;
}

void finish_bf16(ConvW& c) {
  c.b16.resize(c.f32.size());
  for (size_t i = 0; i < c.f32.size(); ++i) c.b16[i] = bf16_rne(c.f32[i]);
}

}  // namespace

Model::~Model() { delete dev; }

void Model::ensure_on_device() {
  std::lock_guard<std::mutex> lk(mu);
  int cur = 0;
  RTE_HIP(hipGetDevice(&cur));
  if (dev) {
    RTE_REQUIRE(device == cur, RTE_EINVAL, "model weights live on another device");
    return;
  }
  DevArena* a = new DevArena();
  try {
    auto up = [&](ConvW& c) {
      c.d32 = a->upload(c.f32);
      c.d16 = a->upload(c.b16);
    };
    for (auto& c : A) up(c);
    for (auto& c : R) up(c);
    for (auto& c : Pr) up(c);
    for (auto& v : Bpre)
      for (auto& c : v) up(c);
    for (auto& v : Bpost)
      for (auto& c : v) up(c);
    for (auto& c : Bc) up(c);
    d_w_in = a->upload(w_in);
    d_w_out = a->upload(w_out);
    {
      const int cq = c0 / 4, dp = slot_budget(ndir);
      std::vector<float> wi(size_t(4) * ndir * cq), wo(size_t(4) * c0 * (dp > 0 ? dp : 0), 0.f);
      for (int sl = 0; sl < 4; ++sl)
        for (int m = 0; m < ndir; ++m)
          for (int q = 0; q < cq; ++q) wi[(size_t(sl) * ndir + m) * cq + q] = w_in[size_t(sl + 4 * q) * ndir + m];
      for (int sl = 0; sl < 4 && dp > 0; ++sl)
        for (int c = 0; c < c0; ++c)
          for (int q = 0; q < dp; ++q) {
            const int m = sl + 4 * q;
            if (m < ndir) wo[(size_t(sl) * c0 + c) * dp + q] = w_out[size_t(m) * c0 + c];
          }
      d_w_in_p = a->upload(wi);
      if (!wo.empty()) d_w_out_p = a->upload(wo);
    }
    for (int l = 0; l < levels; ++l) {
      d_CW.push_back(a->upload(CW[l]));
      d_CB.push_back(a->upload(CB[l]));
      d_HAW.push_back(a->upload(HAW[l]));
      d_HAB.push_back(a->upload(HAB[l]));
      d_HIW.push_back(a->upload(HIW[l]));
      d_HIB.push_back(a->upload(HIB[l]));
    }
  } catch (...) {
    delete a;
    d_CW.clear(); d_CB.clear(); d_HAW.clear(); d_HAB.clear(); d_HIW.clear(); d_HIB.clear();
    throw;
  }
  dev = a;
  device = cur;
}

Model* parse_mgn1(const void* blob, size_t bytes) {
  RTE_REQUIRE(blob != nullptr, RTE_EINVAL, "mgnet_load: null blob");
  const unsigned char* p = static_cast<const unsigned char*>(blob);
  RTE_REQUIRE(bytes >= 48, RTE_EFORMAT, "MGN1: blob shorter than the header");
  RTE_REQUIRE(std::memcmp(p, "MGN1", 4) == 0, RTE_EFORMAT, "MGN1: bad magic");
  RTE_REQUIRE(rd32(p + 4) == 1, RTE_EFORMAT, "MGN1: unsupported version");
  uint32_t h[10];
  for (int i = 0; i < 10; ++i) h[i] = rd32(p + 8 + 4 * i);
  const int dim = int(h[0]), ndir = int(h[1]), c0 = int(h[2]), L = int(h[3]);
  const int nu_pre = int(h[4]), nu_post = int(h[5]), nu_c = int(h[6]), cc = int(h[7]);
  const uint32_t ntens = h[9];
  RTE_REQUIRE(dim == 2 || dim == 3, RTE_EFORMAT, "MGN1: dim must be 2 or 3");
  RTE_REQUIRE(ndir >= 1 && ndir <= 256, RTE_EFORMAT, "MGN1: ndir out of range");
  RTE_REQUIRE(L >= 1 && L <= 8, RTE_EFORMAT, "MGN1: levels out of range");
  RTE_REQUIRE(c0 >= 1 && (int64_t(c0) << (L - 1)) <= 4096, RTE_EFORMAT, "MGN1: channel count out of range");
  RTE_REQUIRE(nu_pre <= 16 && nu_post <= 16 && nu_c <= 16, RTE_EFORMAT, "MGN1: too many smoothing steps");
  RTE_REQUIRE(cc >= 1 && (int64_t(cc) << (L - 1)) <= 4096, RTE_EFORMAT, "MGN1: coef channels out of range");
  RTE_REQUIRE(ntens <= 4096, RTE_EFORMAT, "MGN1: too many tensors");
  RTE_REQUIRE(c0 % 16 == 0, RTE_EINVAL, "mgnet_load: c0 must be a multiple of 16 for the MFMA tiles");

  std::map<uint32_t, Rec> recs;
  size_t off = 48;
  for (uint32_t i = 0; i < ntens; ++i) {
    RTE_REQUIRE(off + 8 <= bytes, RTE_EFORMAT, "MGN1: truncated tensor record");
    uint32_t tag = rd32(p + off), rank = rd32(p + off + 4);
    off += 8;
    RTE_REQUIRE(rank <= 8 && off + 4 * size_t(rank) <= bytes, RTE_EFORMAT, "MGN1: bad rank");
    Rec r;
    size_t cnt = 1;
    for (uint32_t d = 0; d < rank; ++d) {
      uint32_t v = rd32(p + off + 4 * d);
      RTE_REQUIRE(v <= (1u << 24), RTE_EFORMAT, "MGN1: dimension too large");
      r.dims.push_back(v);
      cnt *= v;
      RTE_REQUIRE(cnt <= (size_t(1) << 32), RTE_EFORMAT, "MGN1: tensor too large");
    }
    off += 4 * size_t(rank);
    RTE_REQUIRE(off + 4 * cnt <= bytes, RTE_EFORMAT, "MGN1: truncated tensor data");
    r.data = reinterpret_cast<const float*>(p + off);
    r.count = cnt;
    off += 4 * cnt;
    RTE_REQUIRE(recs.find(tag) == recs.end(), RTE_EFORMAT, "MGN1: duplicate tensor");
    recs[tag] = r;
  }
  RTE_REQUIRE(off == bytes, RTE_EFORMAT, "MGN1: trailing bytes after the last tensor");

  size_t used = 0;
  auto get = [&](int kind, int level, int index, std::vector<uint32_t> shape) {
    uint32_t tag = (uint32_t(kind) << 16) | (uint32_t(level) << 8) | uint32_t(index);
    auto it = recs.find(tag);
    RTE_REQUIRE(it != recs.end(), RTE_EFORMAT,
                "MGN1: missing tensor kind " + std::to_string(kind) + " level " + std::to_string(level) +
                    " index " + std::to_string(index));
    RTE_REQUIRE(it->second.dims == shape, RTE_EFORMAT,
                "MGN1: tensor kind " + std::to_string(kind) + " level " + std::to_string(level) +
                    " has the wrong shape");
    ++used;
    return take(it->second);
  };
  auto kshape = [&](uint32_t a, uint32_t b, int k) {
    std::vector<uint32_t> s{a, b};
    for (int d = 0; d < dim; ++d) s.push_back(uint32_t(k));
    return s;
  };

  Model* m = new Model();
  try {
    m->dim = dim; m->ndir = ndir; m->c0 = c0; m->levels = L;
    m->nu_pre = nu_pre; m->nu_post = nu_post; m->nu_coarse = nu_c; m->coef_ch = cc;
    m->w_in = get(K_WIN, 0, 0, {uint32_t(c0), uint32_t(ndir)});
    m->w_out = get(K_WOUT, 0, 0, {uint32_t(ndir), uint32_t(c0)});
    m->s = get(K_S, 0, 0, {1u})[0];
    m->Bpre.resize(L);
    m->Bpost.resize(L);
    for (int l = 0; l < L; ++l) {
      uint32_t C = uint32_t(c0) << l;
      m->A.push_back(pack_conv3(get(K_A, l, 0, kshape(C, C, 3)), C, C, dim));
      if (l < L - 1) {
        for (int i = 0; i < nu_pre; ++i)
          m->Bpre[l].push_back(pack_conv3(get(K_BPRE, l, i, kshape(C, C, 3)), C, C, dim));
        for (int i = 0; i < nu_post; ++i)
          m->Bpost[l].push_back(pack_conv3(get(K_BPOST, l, i, kshape(C, C, 3)), C, C, dim));
        m->R.push_back(pack_conv3(get(K_R, l, 0, kshape(2 * C, C, 3)), 2 * C, C, dim));
        m->Pr.push_back(pack_convT4(get(K_PR, l, 0, kshape(2 * C, C, 4)), 2 * C, C, dim));
      }
    }
    {
      uint32_t C = uint32_t(c0) << (L - 1);
      for (int i = 0; i < nu_c; ++i)
        m->Bc.push_back(pack_conv3(get(K_BC, L - 1, i, kshape(C, C, 3)), C, C, dim));
    }
    for (int l = 0; l < L; ++l) {
      uint32_t c = uint32_t(cc) << l, cin = l == 0 ? 3u : uint32_t(cc) << (l - 1);
      uint32_t C = uint32_t(c0) << l;
      m->CW.push_back(get(K_CW, l, 0, kshape(c, cin, 3)));
      m->CB.push_back(get(K_CB, l, 0, {c}));
      m->HAW.push_back(get(K_HAW, l, 0, {C, c}));
      m->HAB.push_back(get(K_HAB, l, 0, {C}));
      m->HIW.push_back(get(K_HIW, l, 0, {C, c}));
      m->HIB.push_back(get(K_HIB, l, 0, {C}));
    }
    RTE_REQUIRE(used == recs.size(), RTE_EFORMAT, "MGN1: unexpected extra tensors");
    for (auto& c : m->A) finish_bf16(c);
    for (auto& c : m->R) finish_bf16(c);
    for (auto& c : m->Pr) finish_bf16(c);
    for (auto& v : m->Bpre)
      for (auto& c : v) finish_bf16(c);
    for (auto& v : m->Bpost)
      for (auto& c : v) finish_bf16(c);
    for (auto& c : m->Bc) finish_bf16(c);
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

}  // namespace rte
