// Internal declarations shared by the runtime sources.
#pragma once
#include <stdint.h>

namespace mk {

// Fields of an image in host memory (format v1), after checking the header
// digest, the sizes and the allocation grid. With check_tables the tables
// digest, the kinds and the payload length are checked as well and
// state_digest is filled in.
struct ImageView {
    uint32_t flags = 0, C = 0, n_allocs = 0, base_state = 0, tables_crc = 0, state_digest = 0;
    uint64_t n_chunks = 0, D = 0, N = 0, tl = 0;
    const uint8_t* recs = nullptr;
    const uint8_t* crcs = nullptr;
    const uint8_t* kinds = nullptr;
    const uint8_t* payload = nullptr;
};

int parse_image(const uint8_t* img, uint64_t len, ImageView* v, bool check_tables);

}  // namespace mk
