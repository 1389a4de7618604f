// Files the runtime keeps between processes: the learned cost model with its optimiser state (so
// training resumes where it stopped and a scheduler can start from a trained model), and the GEMM
// tile autotuner's choices (so a process does not re-time every shape).  Both are written to a
// temporary file and renamed into place, carry a 64-bit FNV-1a checksum of their contents, and are
// refused whole -- nothing is applied -- when they are truncated, altered, hold non-finite values
// or were made for another device, runtime or library version.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iterator>
#include <sstream>
#include <string>
#include <vector>

#include "core.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace psc {

namespace {

constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ULL, kFnvPrime = 0x100000001b3ULL;

uint64_t fnv1a64(const void *p, size_t n, uint64_t h = kFnvBasis) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= kFnvPrime;
  }
  return h;
}

std::vector<char> read_file(const std::string &path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) fail(PSC_ERR_IO, "cannot open " + path);
  return std::vector<char>(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
}

void write_file_atomically(const std::string &path, const std::string &bytes) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) fail(PSC_ERR_IO, "cannot create " + tmp);
    f.write(bytes.data(), std::streamsize(bytes.size()));
    f.flush();
    if (!f) fail(PSC_ERR_IO, "cannot write " + tmp);
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    fail(PSC_ERR_IO, "cannot rename " + tmp + " to " + path);
  }
}

// ---- cost-model file ------------------------------------------------------------------------
// Layout (little-endian): magic "PSCMLP01"; uint32 features, hidden units, parameter count, 0;
// int64 Adam step; float32 mean[F], std[F]; float32 params[P], first moments[P], second
// moments[P]; uint64 FNV-1a of every preceding byte.
constexpr char kMlpMagic[8] = {'P', 'S', 'C', 'M', 'L', 'P', '0', '1'};
constexpr size_t kMlpHeader = 8 + 4 * 4 + 8;
constexpr size_t kMlpBody = kMlpHeader + 2 * kMlpF * 4 + 3 * size_t(kMlpP) * 4;
constexpr size_t kMlpFile = kMlpBody + 8;

template <class T>
void put(std::string &out, const T &v) {
  out.append(reinterpret_cast<const char *>(&v), sizeof(T));
}

template <class T>
T get(const char *&p) {
  T v;
  std::memcpy(&v, p, sizeof(T));
  p += sizeof(T);
  return v;
}

}  // namespace

void mlp_file_write(const std::string &path, const MlpState &st) {
  std::string out;
  out.reserve(kMlpFile);
  out.append(kMlpMagic, 8);
  put<uint32_t>(out, uint32_t(kMlpF));
  put<uint32_t>(out, uint32_t(kMlpH));
  put<uint32_t>(out, uint32_t(kMlpP));
  put<uint32_t>(out, 0u);
  put<int64_t>(out, st.step);
  out.append(reinterpret_cast<const char *>(st.mean), kMlpF * 4);
  out.append(reinterpret_cast<const char *>(st.std_), kMlpF * 4);
  for (const std::vector<float> *a : {&st.params, &st.m, &st.v}) {
    if (a->size() != size_t(kMlpP)) fail(PSC_ERR_ARG, "cost-model state of the wrong size");
    out.append(reinterpret_cast<const char *>(a->data()), size_t(kMlpP) * 4);
  }
  put<uint64_t>(out, fnv1a64(out.data(), out.size()));
  write_file_atomically(path, out);
}

MlpState mlp_file_read(const std::string &path) {
  const std::vector<char> b = read_file(path);
  if (b.size() != kMlpFile)
    fail(PSC_ERR_IO, path + ": " + std::to_string(b.size()) + " bytes, a cost-model file has " +
                         std::to_string(kMlpFile) + " (truncated or not such a file)");
  if (std::memcmp(b.data(), kMlpMagic, 8) != 0) fail(PSC_ERR_IO, path + ": not a cost-model file");
  const char *p = b.data() + 8;
  const uint32_t f = get<uint32_t>(p), h = get<uint32_t>(p), np = get<uint32_t>(p);
  (void)get<uint32_t>(p);
  if (f != uint32_t(kMlpF) || h != uint32_t(kMlpH) || np != uint32_t(kMlpP))
    fail(PSC_ERR_IO, path + ": network shape differs from this library's");
  uint64_t want;
  std::memcpy(&want, b.data() + kMlpBody, 8);
  if (fnv1a64(b.data(), kMlpBody) != want) fail(PSC_ERR_IO, path + ": checksum mismatch (file altered or damaged)");
  MlpState st;
  st.step = get<int64_t>(p);
  std::memcpy(st.mean, p, kMlpF * 4);
  p += kMlpF * 4;
  std::memcpy(st.std_, p, kMlpF * 4);
  p += kMlpF * 4;
  for (std::vector<float> *a : {&st.params, &st.m, &st.v}) {
    a->resize(kMlpP);
    std::memcpy(a->data(), p, size_t(kMlpP) * 4);
    p += size_t(kMlpP) * 4;
  }
  if (st.step < 0) fail(PSC_ERR_IO, path + ": negative optimiser step");
  for (int i = 0; i < kMlpF; ++i)
    if (!std::isfinite(st.mean[i]) || !std::isfinite(st.std_[i]) || !(st.std_[i] > 0.0f))
      fail(PSC_ERR_IO, path + ": feature scaling is not finite and positive");
  for (const std::vector<float> *a : {&st.params, &st.m, &st.v})
    for (float v : *a)
      if (!std::isfinite(v)) fail(PSC_ERR_IO, path + ": non-finite parameter or optimiser moment");
  for (float v : st.v)
    if (v < 0.0f) fail(PSC_ERR_IO, path + ": negative second moment");
  return st;
}

// ---- tile-cache file ------------------------------------------------------------------------
// Text: "psc-tile-cache 1", "key <key>", one "entry M N K ab c tile" line per choice, then
// "checksum <16 hex digits>" of every preceding byte.

std::string tile_cache_key(int device) {
  hipDeviceProp_t prop{};
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) fail(PSC_ERR_HIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
  int rt = 0;
  e = hipRuntimeGetVersion(&rt);
  if (e != hipSuccess) fail(PSC_ERR_HIP, std::string("hipRuntimeGetVersion: ") + hipGetErrorString(e));
  const int ntiles = gemm_num_tiles();
  std::string arch = prop.gcnArchName;
  for (char &c : arch)
    if (c == ' ') c = '_';
  return arch + "/cu" + std::to_string(prop.multiProcessorCount) + "/hip" + std::to_string(rt) + "/abi" +
         std::to_string(PSC_ABI_VERSION) + "/tiles" + std::to_string(ntiles);
}

void tile_cache_save(const std::string &path, const std::string &key) {
  if (key.empty() || key.find_first_of(" \n\r\t") != std::string::npos)
    fail(PSC_ERR_ARG, "tile-cache key must be a non-empty word");
  std::ostringstream o;
  o << "psc-tile-cache 1\nkey " << key << "\n";
  for (const auto &e : tile_cache_entries())
    o << "entry " << e[0] << " " << e[1] << " " << e[2] << " " << e[3] << " " << e[4] << " " << e[5] << "\n";
  std::string body = o.str();
  char sum[32];
  std::snprintf(sum, sizeof(sum), "%016llx", static_cast<unsigned long long>(fnv1a64(body.data(), body.size())));
  body += "checksum " + std::string(sum) + "\n";
  write_file_atomically(path, body);
}

int tile_cache_load(const std::string &path, const std::string &key) {
  const std::vector<char> raw = read_file(path);
  const std::string text(raw.begin(), raw.end());
  const size_t cs = text.rfind("checksum ");
  if (cs == std::string::npos || (cs > 0 && text[cs - 1] != '\n')) fail(PSC_ERR_IO, path + ": no checksum line");
  {
    char sum[32];
    std::snprintf(sum, sizeof(sum), "%016llx", static_cast<unsigned long long>(fnv1a64(text.data(), cs)));
    if (text.compare(cs, std::string::npos, "checksum " + std::string(sum) + "\n") != 0)
      fail(PSC_ERR_IO, path + ": checksum mismatch (file altered or damaged)");
  }
  std::istringstream in(text.substr(0, cs));
  std::string line;
  if (!std::getline(in, line) || line != "psc-tile-cache 1") fail(PSC_ERR_IO, path + ": not a tile-cache file");
  if (!std::getline(in, line) || line.rfind("key ", 0) != 0) fail(PSC_ERR_IO, path + ": no key line");
  if (line.substr(4) != key)
    fail(PSC_ERR_STATE, path + ": made for " + line.substr(4) + ", not for " + key + " (nothing loaded)");
  std::vector<std::array<int, 6>> got;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string w;
    std::array<int, 6> e{};
    if (!(ls >> w) || w != "entry") fail(PSC_ERR_IO, path + ": unexpected line '" + line + "'");
    for (int &v : e)
      if (!(ls >> v)) fail(PSC_ERR_IO, path + ": short entry '" + line + "'");
    if (ls >> w) fail(PSC_ERR_IO, path + ": long entry '" + line + "'");
    if (e[0] < 0 || e[1] < 0 || e[2] < 0 || (e[3] != PSC_F32 && e[3] != PSC_BF16) ||
        (e[4] != PSC_F32 && e[4] != PSC_BF16) || e[5] < 1 || e[5] >= gemm_num_tiles())
      fail(PSC_ERR_IO, path + ": entry out of range '" + line + "'");
    got.push_back(e);
  }
  for (const auto &e : got) tile_cache_set(e[0], e[1], e[2], e[3], e[4], e[5]);
  return int(got.size());
}

}  // namespace psc
