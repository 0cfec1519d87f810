// Serving runtime of libtersoff.so: many independent configurations evaluated
// in batches (declarations shared by tersoff_api.hip and serve.hip; the C ABI
// is in include/tersoff.h).
#pragma once

#include "internal.h"
#include "tersoff.h"

#include <string>

namespace tsf {

struct Server;

// Context data the server reads (the parameter table stays owned by the
// context, which outlives the server).
struct ServerEnv {
    int device;
    int ntypes;
    double max_cut;
    DeviceTable tab;
};

int server_create(const ServerEnv &env, const tersoff_serve_config &cfg, Server **out, std::string &err);
// Finishes every queued and in-flight request, then joins the worker.
void server_destroy(Server *s);
int server_submit(Server *s, const tersoff_request &req, uint64_t *ticket, std::string &err);
int server_poll(Server *s, uint64_t ticket, tersoff_result *res, double timeout_ms, std::string &err);
void server_stats(Server *s, double out[6]);

}  // namespace tsf
