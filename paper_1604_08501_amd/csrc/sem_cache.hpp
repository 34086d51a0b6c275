// Plan cache file of the mixed-order batch autotuner: a flat JSON object
// {"key": {"epb": E, "layout": L, "us": T}, ...}.  Host-only C++ (no HIP),
// internal to libsem.so; kept in a translation unit of its own so that the
// reader can be exercised on malformed files by a sanitizer build on the CPU.
#pragma once
#include <map>
#include <string>

namespace semcache {

struct Entry {
    int epb = 0;
    int lay = 0;
    double us = -1.0;
};

// Entries of the file at `path` (empty if it is missing or unreadable).
// Malformed text yields fewer entries, never undefined behaviour: numbers are
// accepted only when finite and within range (epb 1..4096, layout 0..15,
// us >= 0), keys only up to 256 characters.
std::map<std::string, Entry> read(const std::string& path);

// Writes `m` to path + ".tmp" and renames it over `path`.
void write(const std::string& path, const std::map<std::string, Entry>& m);

}  // namespace semcache
