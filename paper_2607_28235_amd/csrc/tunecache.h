// Persisted cache of the library's kernel timings (host side).
//
// The kernel choices made by timing (the fine level's single-right-hand-side row-block shape at set-up, the
// multi-right-hand-side kernel of every level and of PCG's operator at the first solve with that many columns)
// depend on the device, on the level structure and on the precision, not on the numeric values.  They are kept in
// a text file, one "key value" line per choice, so that a later handle of the same structure (in this process or
// another) skips the timing.  The file is R3MG_TUNE_CACHE if that environment variable is set (an empty value:
// no file), else $HOME/.cache/r3mg/tune-cache.txt.  It is re-read at each lookup and extended with one appended
// line per new choice (a single write, so that processes sharing the file do not interleave lines); malformed
// lines are ignored, and the last line of a key wins.  A file that cannot be read or written only means that the
// choice is timed again.
#pragma once

#include <cstdint>
#include <string>

namespace r3mg {

// version of the kernel set the cached codes refer to (bump when shapes or codes change meaning)
constexpr int kTuneCacheVersion = 2;

// key prefix naming the device (architecture, compute units) and the tuning version
std::string tune_device_key(int dev);

// value cached under key, or false
bool tune_cache_get(const std::string& key, int* value);
// records value under key (appends a line; errors are ignored)
void tune_cache_put(const std::string& key, int value);

// 64-bit FNV-1a over a byte range, continued from h
uint64_t fnv1a(const void* data, size_t bytes, uint64_t h = 1469598103934665603ull);

}  // namespace r3mg
