// JSON cache of tuned choices (see json_cache.hpp).
#include "json_cache.hpp"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

namespace dg {

std::map<std::string, std::string> read_cache(const std::string& path) {
  std::map<std::string, std::string> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = s.find("\"entries\"");
  if (pos == std::string::npos) return out;
  pos = s.find('{', pos);
  if (pos == std::string::npos) return out;
  ++pos;
  for (;;) {
    const size_t k0 = s.find_first_of("\"}", pos);
    if (k0 == std::string::npos || s[k0] == '}') break;
    const size_t k1 = s.find('"', k0 + 1);
    if (k1 == std::string::npos) break;
    const size_t o0 = s.find('{', k1);
    const size_t o1 = o0 == std::string::npos ? o0 : s.find('}', o0);
    if (o1 == std::string::npos) break;
    out[s.substr(k0 + 1, k1 - k0 - 1)] = s.substr(o0, o1 - o0 + 1);
    pos = o1 + 1;
  }
  return out;
}

bool cache_field(const std::string& obj, const char* name, double& v) {
  const std::string pat = std::string("\"") + name + "\"";
  const size_t p = obj.find(pat);
  if (p == std::string::npos) return false;
  const size_t c = obj.find(':', p + pat.size());
  if (c == std::string::npos) return false;
  char* end = nullptr;
  v = std::strtod(obj.c_str() + c + 1, &end);
  return end != obj.c_str() + c + 1;
}

bool write_cache(const std::string& path, const std::map<std::string, std::string>& entries) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{\n  \"version\": 1,\n  \"entries\": {";
    bool first = true;
    for (const auto& kv : entries) {
      f << (first ? "\n" : ",\n") << "    \"" << kv.first << "\": " << kv.second;
      first = false;
    }
    f << "\n  }\n}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}


std::string device_key(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + ":" + std::to_string(prop.multiProcessorCount) + "cu";
}

}  // namespace dg
