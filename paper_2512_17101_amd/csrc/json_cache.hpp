// Tiny JSON file of tuned choices shared by the autotuners:
//   {"version": 1, "entries": {"<key>": {"name": number, ...}, ...}}
// (flat objects of numbers only; written atomically via a temporary file).
#pragma once
#include <map>
#include <string>

namespace dg {

// Every "key": {object} pair of the "entries" object, objects kept as text;
// empty if the file is missing or unreadable.
std::map<std::string, std::string> read_cache(const std::string& path);
// Number stored under "name" in a flat object's text.
bool cache_field(const std::string& obj, const char* name, double& v);
bool write_cache(const std::string& path, const std::map<std::string, std::string>& entries);
// "<arch>:<CUs>cu" of a device, the prefix of every key.
std::string device_key(int device);

}  // namespace dg
