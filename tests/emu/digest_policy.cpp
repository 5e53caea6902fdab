// The resident digest tables' eviction rule (runtime.h digest_victim) over
// the context's own entry type, for a CPU test: a table pinned by a request
// in flight must never be chosen.
#include <stdint.h>

#include <unordered_map>

#include "runtime.h"

extern "C" uint64_t emu_digest_victim(const uint64_t* uids, const uint64_t* last_use, const uint32_t* pins, int n) {
    std::unordered_map<uint64_t, mk::DigestEntry> m;
    for (int i = 0; i < n; ++i) {
        mk::DigestEntry& e = m[uids[i]];
        e.last_use = last_use[i];
        e.pins = pins[i];
    }
    return mk::digest_victim(m, 0);
}
