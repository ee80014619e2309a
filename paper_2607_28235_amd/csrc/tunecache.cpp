// Persisted cache of the library's kernel timings (see tunecache.h).
#include "tunecache.h"

#include <hip/hip_runtime.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fcntl.h>
#include <mutex>
#include <sys/stat.h>
#include <unistd.h>

namespace r3mg {

namespace {

std::mutex g_mu;

// the cache file ("" = none)
std::string cache_path() {
  if (const char* e = std::getenv("R3MG_TUNE_CACHE")) return std::string(e);
  const char* home = std::getenv("HOME");
  if (!home || !*home) return std::string();
  return std::string(home) + "/.cache/r3mg/tune-cache.txt";
}

// creates the directories above path (best effort)
void make_parents(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') {
      const std::string d = path.substr(0, i);
      if (::mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return;
    }
}

}  // namespace

uint64_t fnv1a(const void* data, size_t bytes, uint64_t h) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string tune_device_key(int dev) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  } else {
    (void)hipGetLastError();
  }
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  return "v" + std::to_string(kTuneCacheVersion) + "/" + arch + "/" + std::to_string(cus) + "cu";
}

bool tune_cache_get(const std::string& key, int* value) {
  const std::string path = cache_path();
  if (path.empty()) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  bool found = false;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const size_t len = std::strlen(line);
    if (len == 0 || line[len - 1] != '\n') continue;  // truncated or partial line
    char* sp = std::strrchr(line, ' ');
    if (!sp) continue;
    *sp = '\0';
    if (key != line) continue;
    char* end = nullptr;
    const long v = std::strtol(sp + 1, &end, 10);
    if (end == sp + 1 || (*end != '\n' && *end != '\0')) continue;
    *value = (int)v;
    found = true;  // the last line of the key wins
  }
  std::fclose(f);
  return found;
}

void tune_cache_put(const std::string& key, int value) {
  const std::string path = cache_path();
  if (path.empty() || key.find('\n') != std::string::npos) return;
  std::lock_guard<std::mutex> lk(g_mu);
  make_parents(path);
  const int fd = ::open(path.c_str(), O_WRONLY | O_CREAT | O_APPEND, 0644);
  if (fd < 0) return;
  const std::string line = key + " " + std::to_string(value) + "\n";
  (void)!::write(fd, line.data(), line.size());
  ::close(fd);
}

}  // namespace r3mg
