// Checkpoints of the learned preconditioner's parameter vector, in the safetensors layout:
//   8 bytes   little-endian length L of the header
//   L bytes   JSON header: {"__metadata__": {string: string, ...},
//                           "params": {"dtype": "F32", "shape": [n], "data_offsets": [0, 4 n]}}
//   4 n bytes the FP32 parameters (little-endian), in the order of hdg_gnn_param_count.
// The shape of the network is kept in the metadata as "d2", "hidden" and "layers".  Host
// code only: the caller moves the parameters between host and device memory.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hdg_internal.h"

namespace hdg {
namespace {

// ---- a small JSON reader for the header (objects, arrays, strings, numbers)
struct Json {
  enum Kind { NUL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<Json> arr;
  std::map<std::string, Json> obj;
};

struct Parser {
  const char* p;
  const char* end;
  bool ok = true;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool eat(char c) {
    ws();
    if (p < end && *p == c) {
      ++p;
      return true;
    }
    return false;
  }
  std::string string() {
    std::string out;
    if (!eat('"')) {
      ok = false;
      return out;
    }
    while (p < end && *p != '"') {
      char c = *p++;
      if (c == '\\' && p < end) {
        const char e = *p++;
        switch (e) {
          case 'n': c = '\n'; break;
          case 't': c = '\t'; break;
          case 'r': c = '\r'; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'u': {  // only the ASCII range is expected in these headers
            unsigned v = 0;
            for (int i = 0; i < 4 && p < end; ++i, ++p) {
              const char h = *p;
              v = v * 16 + (h >= '0' && h <= '9' ? h - '0' : (h | 32) - 'a' + 10);
            }
            c = v < 128 ? (char)v : '?';
            break;
          }
          default: c = e;
        }
      }
      out.push_back(c);
    }
    if (p >= end) ok = false;
    ++p;
    return out;
  }
  Json value(int depth = 0) {
    Json j;
    ws();
    if (p >= end || depth > 16) {
      ok = false;
      return j;
    }
    if (*p == '{') {
      ++p;
      j.kind = Json::OBJ;
      if (eat('}')) return j;
      do {
        std::string k = string();
        if (!eat(':')) {
          ok = false;
          return j;
        }
        j.obj[k] = value(depth + 1);
      } while (ok && eat(','));
      if (!eat('}')) ok = false;
    } else if (*p == '[') {
      ++p;
      j.kind = Json::ARR;
      if (eat(']')) return j;
      do j.arr.push_back(value(depth + 1));
      while (ok && eat(','));
      if (!eat(']')) ok = false;
    } else if (*p == '"') {
      j.kind = Json::STR;
      j.str = string();
    } else {
      char* q = nullptr;
      j.num = std::strtod(p, &q);
      if (q == p) ok = false;
      j.kind = Json::NUM;
      p = q;
    }
    return j;
  }
};

std::string quote(const std::string& s) {
  std::string o = "\"";
  for (char c : s) {
    if (c == '"' || c == '\\') {
      o.push_back('\\');
      o.push_back(c);
    } else if ((unsigned char)c < 0x20) {
      char b[8];
      std::snprintf(b, sizeof b, "\\u%04x", (unsigned)(unsigned char)c);
      o += b;
    } else {
      o.push_back(c);
    }
  }
  return o + "\"";
}

struct Checkpoint {
  Json header;
  size_t data_begin = 0;
  int64_t n = 0;
};

hdg_status read_header(const char* path, Checkpoint& ck, const char* who) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": cannot open " + path);
  unsigned char lb[8];
  if (std::fread(lb, 1, 8, f) != 8) {
    std::fclose(f);
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": truncated file");
  }
  uint64_t len = 0;
  for (int i = 7; i >= 0; --i) len = len << 8 | lb[i];
  if (len == 0 || len > (1u << 26)) {
    std::fclose(f);
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": bad header length");
  }
  std::string h(len, '\0');
  const size_t got = std::fread(&h[0], 1, len, f);
  std::fclose(f);
  if (got != len) return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": truncated header");
  Parser ps{h.data(), h.data() + h.size()};
  ck.header = ps.value();
  if (!ps.ok || ck.header.kind != Json::OBJ)
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": header is not a JSON object");
  auto it = ck.header.obj.find("params");
  if (it == ck.header.obj.end() || it->second.kind != Json::OBJ)
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": no tensor named params");
  const Json& t = it->second;
  auto dt = t.obj.find("dtype");
  auto sh = t.obj.find("shape");
  auto off = t.obj.find("data_offsets");
  if (dt == t.obj.end() || dt->second.str != "F32" || sh == t.obj.end() || sh->second.arr.size() != 1 ||
      off == t.obj.end() || off->second.arr.size() != 2)
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": params must be a 1-D F32 tensor");
  ck.n = (int64_t)sh->second.arr[0].num;
  const int64_t b0 = (int64_t)off->second.arr[0].num, b1 = (int64_t)off->second.arr[1].num;
  if (ck.n < 1 || b1 - b0 != 4 * ck.n || b0 < 0)
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": inconsistent params entry");
  ck.data_begin = 8 + (size_t)len + (size_t)b0;
  return HDG_OK;
}

const std::string* meta(const Checkpoint& ck, const char* key) {
  auto m = ck.header.obj.find("__metadata__");
  if (m == ck.header.obj.end() || m->second.kind != Json::OBJ) return nullptr;
  auto v = m->second.obj.find(key);
  if (v == m->second.obj.end() || v->second.kind != Json::STR) return nullptr;
  return &v->second.str;
}

}  // namespace
}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_gnn_save(const char* path, const hdg_gnn_shape* shape, const float* h_params, int64_t n,
                                   const char* const* meta_keys, const char* const* meta_values, int nmeta) {
  if (!path || !shape || !h_params || n < 1 || nmeta < 0 || (nmeta > 0 && (!meta_keys || !meta_values)))
    return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_save: bad argument");
  int64_t need = 0;
  hdg_status st = hdg_gnn_param_count(shape, &need);
  if (st) return st;
  if (need != n) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_save: parameter count does not match the shape");
  std::map<std::string, std::string> md;
  for (int i = 0; i < nmeta; ++i) {
    if (!meta_keys[i] || !meta_values[i]) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_save: NULL metadata");
    md[meta_keys[i]] = meta_values[i];
  }
  md["d2"] = std::to_string(shape->d2);
  md["hidden"] = std::to_string(shape->hidden);
  md["layers"] = std::to_string(shape->layers);
  std::string h = "{\"__metadata__\":{";
  bool first = true;
  for (const auto& kv : md) {
    if (!first) h += ",";
    first = false;
    h += quote(kv.first) + ":" + quote(kv.second);
  }
  h += "},\"params\":{\"dtype\":\"F32\",\"shape\":[" + std::to_string(n) + "],\"data_offsets\":[0," +
       std::to_string(4 * n) + "]}}";
  while (h.size() % 8) h.push_back(' ');  // the data start stays 8-byte aligned
  FILE* f = std::fopen(path, "wb");
  if (!f) return set_error(HDG_ERR_INVALID_ARG, std::string("hdg_gnn_save: cannot create ") + path);
  unsigned char lb[8];
  uint64_t len = h.size();
  for (int i = 0; i < 8; ++i) lb[i] = (unsigned char)(len >> (8 * i));
  bool ok = std::fwrite(lb, 1, 8, f) == 8 && std::fwrite(h.data(), 1, h.size(), f) == h.size();
  for (int64_t i = 0; ok && i < n; ++i) {  // little-endian FP32 words, independent of the host order
    uint32_t u;
    std::memcpy(&u, h_params + i, 4);
    const unsigned char w[4] = {(unsigned char)u, (unsigned char)(u >> 8), (unsigned char)(u >> 16),
                                (unsigned char)(u >> 24)};
    ok = std::fwrite(w, 1, 4, f) == 4;
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return set_error(HDG_ERR_INVALID_ARG, std::string("hdg_gnn_save: write failed for ") + path);
  return HDG_OK;
}

extern "C" hdg_status hdg_gnn_load_info(const char* path, hdg_gnn_shape* shape, int64_t* n) {
  if (!path || !shape || !n) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_load_info: NULL argument");
  Checkpoint ck;
  hdg_status st = read_header(path, ck, "hdg_gnn_load_info");
  if (st) return st;
  const std::string *d2 = meta(ck, "d2"), *h = meta(ck, "hidden"), *l = meta(ck, "layers");
  if (!d2 || !h || !l) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_load_info: shape missing from the metadata");
  shape->d2 = std::atoi(d2->c_str());
  shape->hidden = std::atoi(h->c_str());
  shape->layers = std::atoi(l->c_str());
  int64_t need = 0;
  st = hdg_gnn_param_count(shape, &need);
  if (st) return st;
  if (need != ck.n) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_load_info: parameter count does not match the shape");
  *n = ck.n;
  return HDG_OK;
}

extern "C" hdg_status hdg_gnn_load(const char* path, float* h_params, int64_t n) {
  if (!path || !h_params || n < 1) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_load: bad argument");
  Checkpoint ck;
  hdg_status st = read_header(path, ck, "hdg_gnn_load");
  if (st) return st;
  if (ck.n != n) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_load: parameter count differs from the file's");
  FILE* f = std::fopen(path, "rb");
  if (!f) return set_error(HDG_ERR_INVALID_ARG, std::string("hdg_gnn_load: cannot open ") + path);
  bool ok = std::fseek(f, (long)ck.data_begin, SEEK_SET) == 0;
  for (int64_t i = 0; ok && i < n; ++i) {
    unsigned char w[4];
    ok = std::fread(w, 1, 4, f) == 4;
    const uint32_t u = (uint32_t)w[0] | (uint32_t)w[1] << 8 | (uint32_t)w[2] << 16 | (uint32_t)w[3] << 24;
    std::memcpy(h_params + i, &u, 4);
  }
  std::fclose(f);
  if (!ok) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_load: truncated data");
  return HDG_OK;
}

extern "C" hdg_status hdg_gnn_checkpoint_meta(const char* path, const char* key, char* out, size_t cap, size_t* len) {
  if (!path || !key || !len) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_checkpoint_meta: NULL argument");
  Checkpoint ck;
  hdg_status st = read_header(path, ck, "hdg_gnn_checkpoint_meta");
  if (st) return st;
  const std::string* v = meta(ck, key);
  if (!v) return set_error(HDG_ERR_INVALID_ARG, std::string("hdg_gnn_checkpoint_meta: no key ") + key);
  *len = v->size();
  if (out && cap > 0) {
    const size_t m = std::min(cap - 1, v->size());
    std::memcpy(out, v->data(), m);
    out[m] = '\0';
  }
  return HDG_OK;
}
