// Request server internals (serve.hip); the C ABI wraps them.
#pragma once

#include "rte_internal.h"

namespace rte {

struct Server;
void mesh_init(Mesh &M, const rte_mesh_desc_t &d);
Server *server_create(const rte_server_desc_t &d, hipStream_t s);
void server_destroy(Server *S);
int server_add_mesh(Server &S, const rte_mesh_desc_t &md, const double *kappa);
int64_t server_submit(Server &S, const rte_request_t &q);
void server_step(Server &S, int32_t *n_active, int32_t *n_pending);
void server_poll(Server &S, int64_t id, rte_request_info_t &info);
void server_levels(Server &S, int64_t id, int32_t *levels);
void server_fetch(Server &S, int64_t id, double *T_out);
int64_t server_mesh_size(Server &S, int mesh, int64_t *L);
rte_server_stats_t server_stats(Server &S);

}  // namespace rte

struct rte_server { rte::Server *srv = nullptr; };
