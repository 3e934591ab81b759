// The set-up's sparse product C = A B on the device, equal bit for bit to the
// host product spgemm (host_csr.hpp).
#pragma once

#include "host_csr.hpp"

namespace mdp {

// stream: a hipStream_t.  Returns false, leaving c untouched, when the
// product is empty, too large for the device buffers (more than 2^29 terms)
// or the device memory for it cannot be allocated; the caller then forms it
// on the host.  Other device errors throw.
bool device_spgemm(const HCsr &a, const HCsr &b, HCsr &c, void *stream);

}  // namespace mdp
