// Host-side model object behind the opaque cbvh_model handle.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "format.h"

struct cbvh_model {
    std::vector<uint8_t> blob;  // serialized model, exactly what is uploaded
    cbvh::BlobHeader hdr;       // parsed copy of the header
    uint32_t n_inner = 0, n_leaves = 0;
    uint64_t descriptor_bytes = 0;
};

namespace cbvh {

struct BuildParams {
    uint32_t bv, branching, leaf_size, bits, treelet_bytes;
};

// Builds the blob into m->blob and fills m->hdr.  Returns an empty string on
// success, else a message (the caller maps it to CBVH_E_INVALID).
std::string build_model(const float *V, uint32_t nv, const uint32_t *T, uint32_t nt, const BuildParams &p,
                        cbvh_model *m);

// Validates a serialized model (header, sections, topology, index ranges).
// Returns an empty string if the blob is safe to traverse on the device.
std::string validate_blob(const uint8_t *blob, size_t n, BlobHeader *hdr, uint32_t *n_inner, uint32_t *n_leaves);

}  // namespace cbvh
