// server.cpp -- continuous-batching request server (filled in below).
#include "runtime.h"

extern "C" {
int ising_server_create(uint64_t, int32_t, int32_t, int32_t, void*, ising_server**) { return ISING_ERR_UNSUPPORTED; }
int ising_server_submit(ising_server*, ising_problem*, const ising_schedule*, int32_t, uint64_t, int64_t, int32_t, uint64_t*) { return ISING_ERR_UNSUPPORTED; }
int ising_server_wait(ising_server*, uint64_t, double, ising_result*) { return ISING_ERR_UNSUPPORTED; }
int ising_server_best_state(ising_server*, uint64_t, int8_t*) { return ISING_ERR_UNSUPPORTED; }
int ising_server_footprint(const ising_problem*, const ising_schedule*, int32_t, uint64_t*) { return ISING_ERR_UNSUPPORTED; }
int ising_server_stats(ising_server*, int64_t*, int64_t*, int32_t*) { return ISING_ERR_UNSUPPORTED; }
int ising_server_destroy(ising_server*) { return ISING_OK; }
}
