// Weight file of the collocation network H ("SL7W" version 1, little endian):
//   char[4] "SL7W"; u32 version; u32 d_in, width, depth, m, act, model;
//   f64 in_scale[d_in], in_shift[d_in], dom_lo[d_in], dom_hi[d_in];
//   per layer l = 0..depth: f32 W_l[out * in] (row-major), f32 b_l[out];
//   u32 meta_len; meta_len bytes of UTF-8 JSON.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sl7_host.hpp"

using namespace sl7;

namespace {

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

bool read_all(const char* path, std::vector<unsigned char>& out) {
  File F;
  F.f = fopen(path, "rb");
  if (!F.f) return false;
  unsigned char buf[1 << 16];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), F.f)) > 0) out.insert(out.end(), buf, buf + n);
  return !ferror(F.f);
}

template <class T>
bool take(const std::vector<unsigned char>& d, size_t& off, T* dst, size_t count) {
  const size_t n = sizeof(T) * count;
  if (off + n > d.size()) return false;
  std::memcpy(dst, d.data() + off, n);
  off += n;
  return true;
}

}  // namespace

extern "C" int sl7_mlp_load(const char* path, sl7_mlp** out) {
  if (!path || !out) return fail(SL7_EINVAL, "path and H must be non-NULL");
  *out = nullptr;
  std::vector<unsigned char> d;
  if (!read_all(path, d)) return fail(SL7_EIO, "cannot read %s", path);
  size_t off = 0;
  char magic[4];
  uint32_t hdr[7];
  if (!take(d, off, magic, 4) || std::memcmp(magic, "SL7W", 4) != 0)
    return fail(SL7_EINVAL, "%s: bad magic", path);
  if (!take(d, off, hdr, 7)) return fail(SL7_EINVAL, "%s: truncated header", path);
  if (hdr[0] != 1) return fail(SL7_EINVAL, "%s: unsupported version %u", path, hdr[0]);
  sl7_mlp_desc desc;
  std::memset(&desc, 0, sizeof(desc));
  desc.d_in = (int)hdr[1];
  desc.width = (int)hdr[2];
  desc.depth = (int)hdr[3];
  desc.m = (int)hdr[4];
  desc.act = (int)hdr[5];
  desc.model = (int)hdr[6];
  if (desc.d_in < 1 || desc.d_in > SL7_MAX_DIN) return fail(SL7_EINVAL, "%s: d_in=%d out of range", path, desc.d_in);
  if (!take(d, off, desc.in_scale, desc.d_in) || !take(d, off, desc.in_shift, desc.d_in) ||
      !take(d, off, desc.dom_lo, desc.d_in) || !take(d, off, desc.dom_hi, desc.d_in))
    return fail(SL7_EINVAL, "%s: truncated input affine", path);
  int rc = check_desc(&desc);
  if (rc) return rc;
  std::vector<float> params((size_t)n_params_of(desc));
  if (!take(d, off, params.data(), params.size())) return fail(SL7_EINVAL, "%s: truncated weights", path);
  uint32_t meta_len = 0;
  std::string meta;
  if (take(d, off, &meta_len, 1)) {
    if (off + meta_len > d.size()) return fail(SL7_EINVAL, "%s: truncated metadata", path);
    meta.assign((const char*)d.data() + off, meta_len);
  }
  sl7_mlp* H = nullptr;
  rc = sl7_mlp_create(&desc, params.data(), &H);
  if (rc) return rc;
  reinterpret_cast<Mlp*>(H)->meta = meta;
  *out = H;
  return SL7_OK;
}

extern "C" int sl7_mlp_save(const sl7_mlp* Hc, const char* path) {
  if (!Hc || !path) return fail(SL7_EINVAL, "H and path must be non-NULL");
  const Mlp* H = reinterpret_cast<const Mlp*>(Hc);
  File F;
  F.f = fopen(path, "wb");
  if (!F.f) return fail(SL7_EIO, "cannot open %s for writing", path);
  const uint32_t hdr[7] = {1u, (uint32_t)H->d.d_in, (uint32_t)H->d.width, (uint32_t)H->d.depth,
                           (uint32_t)H->d.m, (uint32_t)H->d.act, (uint32_t)H->d.model};
  const uint32_t meta_len = (uint32_t)H->meta.size();
  bool ok = fwrite("SL7W", 1, 4, F.f) == 4 && fwrite(hdr, 4, 7, F.f) == 7 &&
            fwrite(H->d.in_scale, 8, H->d.d_in, F.f) == (size_t)H->d.d_in &&
            fwrite(H->d.in_shift, 8, H->d.d_in, F.f) == (size_t)H->d.d_in &&
            fwrite(H->d.dom_lo, 8, H->d.d_in, F.f) == (size_t)H->d.d_in &&
            fwrite(H->d.dom_hi, 8, H->d.d_in, F.f) == (size_t)H->d.d_in &&
            fwrite(H->params.data(), 4, H->params.size(), F.f) == H->params.size() &&
            fwrite(&meta_len, 4, 1, F.f) == 1 &&
            (meta_len == 0 || fwrite(H->meta.data(), 1, meta_len, F.f) == meta_len);
  if (!ok) return fail(SL7_EIO, "write to %s failed", path);
  return SL7_OK;
}
