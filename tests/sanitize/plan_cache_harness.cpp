// Drives the plan-cache reader and writer (paper_1604_08501_amd/csrc/
// sem_cache.cpp) over the files named on the command line, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer: every file is read, every
// entry is checked against the documented ranges, and the entries are
// written and read back unchanged.  Exit status 0 when all checks hold.
#include <cstdio>
#include <string>

#include "sem_cache.hpp"

int main(int argc, char** argv)
{
    if (argc < 3) {
        fprintf(stderr, "usage: %s SCRATCH_FILE CACHE_FILE...\n", argv[0]);
        return 2;
    }
    const std::string scratch = argv[1];
    for (int a = 2; a < argc; ++a) {
        const auto m = semcache::read(argv[a]);
        for (const auto& kv : m) {
            const semcache::Entry& e = kv.second;
            if (kv.first.size() > 256 || e.epb < 1 || e.epb > 4096 || e.lay < 0 || e.lay > 15 ||
                !(e.us >= 0.0)) {
                fprintf(stderr, "%s: entry out of range\n", argv[a]);
                return 1;
            }
        }
        semcache::write(scratch, m);
        const auto back = semcache::read(scratch);
        if (back.size() != m.size()) {
            fprintf(stderr, "%s: %zu entries written, %zu read back\n", argv[a], m.size(),
                    back.size());
            return 1;
        }
        for (const auto& kv : m) {
            auto it = back.find(kv.first);
            if (it == back.end() || it->second.epb != kv.second.epb ||
                it->second.lay != kv.second.lay) {
                fprintf(stderr, "%s: entry %s changed on the round trip\n", argv[a],
                        kv.first.c_str());
                return 1;
            }
        }
        printf("%s: %zu entries\n", argv[a], m.size());
    }
    return 0;
}
