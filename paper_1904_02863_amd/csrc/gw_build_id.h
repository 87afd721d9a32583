// Identity of the sources each translation unit was compiled from.  The
// build passes GW_SOURCE_HASH (SHA-256 over the library's sources and its
// public header) to every compile, and each translation unit reports it under
// a name of its own, so that the library can tell when it has been linked
// from objects of different builds (whose internal structures need not
// agree) and refuse to run.
#pragma once

#ifndef GW_SOURCE_HASH
#define GW_SOURCE_HASH "unknown"
#endif

namespace gw {
const char *source_hash_api();
const char *source_hash_kernels();
const char *source_hash_flow();
const char *source_hash_mcmc();
const char *source_hash_pop();
const char *source_hash_relbin();
const char *source_hash_waveform();
// GW_OK when every translation unit reports the same hash, else GW_EABI
// (with the message of gw_last_error set).
int check_build();
}  // namespace gw

#define GW_DEFINE_SOURCE_HASH(unit) \
    namespace gw {                  \
    const char *source_hash_##unit() { return GW_SOURCE_HASH; } \
    }
