// The method table of smmo_parallel_do(): method name (smmo_method_id), the
// size of its argument struct and its launcher.  Method ids are indices into
// this table and part of the ABI's behaviour (smmo_method_id resolves names).
#include <hip/hip_runtime.h>

#include "../../include/smmo_methods.h"
#include "method_common.hpp"

namespace smmo {

// launchers of the method table: methods.hip
smmo_status launch_gol_cell_count(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_gol_alive_death(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_gol_cell_birth(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_gol_generation(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_nbody_force(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_nbody_update(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_test_axpy(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_test_destroy_if(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_test_spawn(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_test_transmute(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_ls_alloc(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_ls_free(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);

// launchers defined in spring.hip
smmo_status launch_spring_force(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_spring_node_update(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_spring_link(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);

// launchers defined in spring_pi.hip
smmo_status launch_spring_pi_force(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_spring_pi_node_update(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_spring_pi_link(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);

// launchers defined in generation.hip
smmo_status launch_generation_cell_count(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_generation_cell_birth(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_generation_alive_update(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);

// launchers defined in structure.hip
smmo_status launch_structure_pull(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_structure_force(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_structure_node_update(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_structure_bfs_init(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_structure_bfs_visit(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_structure_bfs_mark(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_structure_bfs_delete(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_structure_link(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);

// launchers defined in adjoint.hip
smmo_status launch_adj_record(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_adj_step_node(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_adj_save(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_adj_load(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_adj_seed(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_adj_zero(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_adj_node(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_adj_spring(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);

// launchers defined in wator.hip
smmo_status launch_wator_cell_prepare(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_wator_fish_prepare(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_wator_shark_prepare(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_wator_cell_decide(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_wator_fish_update(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_wator_shark_update(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_wator_cell_link(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
smmo_status launch_wator_link(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);

namespace {
const MethodEntry kMethods[] = {
    {"gol.cell_count", sizeof(smmo_gol_args), launch_gol_cell_count},
    {"gol.alive_death", sizeof(smmo_gol_args), launch_gol_alive_death},
    {"gol.cell_birth", sizeof(smmo_gol_args), launch_gol_cell_birth},
    {"nbody.force", sizeof(smmo_nbody_args), launch_nbody_force},
    {"nbody.update", sizeof(smmo_nbody_args), launch_nbody_update},
    {"spring.force", sizeof(smmo_spring_args), launch_spring_force},
    {"spring.node_update", sizeof(smmo_spring_args), launch_spring_node_update},
    {"spring.link", sizeof(smmo_spring_args), launch_spring_link},
    {"adjoint.record", sizeof(smmo_adjoint_args), launch_adj_record},
    {"adjoint.save", sizeof(smmo_adjoint_args), launch_adj_save},
    {"adjoint.load", sizeof(smmo_adjoint_args), launch_adj_load},
    {"adjoint.seed", sizeof(smmo_adjoint_args), launch_adj_seed},
    {"adjoint.zero", sizeof(smmo_adjoint_args), launch_adj_zero},
    {"adjoint.node", sizeof(smmo_adjoint_args), launch_adj_node},
    {"adjoint.spring", sizeof(smmo_adjoint_args), launch_adj_spring},
    {"adjoint.step_node", sizeof(smmo_adjoint_args), launch_adj_step_node},
    {"test.axpy", sizeof(smmo_axpy_args), launch_test_axpy},
    {"test.destroy_if", sizeof(smmo_destroy_if_args), launch_test_destroy_if},
    {"test.spawn", sizeof(smmo_spawn_args), launch_test_spawn},
    {"test.transmute", sizeof(smmo_spawn_args), launch_test_transmute},
    {"alloc.ls_alloc", sizeof(smmo_ls_args), launch_ls_alloc},
    {"alloc.ls_free", sizeof(smmo_ls_args), launch_ls_free},
    {"wator.cell_prepare", sizeof(smmo_wator_args), launch_wator_cell_prepare},
    {"wator.fish_prepare", sizeof(smmo_wator_args), launch_wator_fish_prepare},
    {"wator.shark_prepare", sizeof(smmo_wator_args), launch_wator_shark_prepare},
    {"wator.cell_decide", sizeof(smmo_wator_args), launch_wator_cell_decide},
    {"wator.fish_update", sizeof(smmo_wator_args), launch_wator_fish_update},
    {"wator.shark_update", sizeof(smmo_wator_args), launch_wator_shark_update},
    {"wator.cell_link", sizeof(smmo_wator_args), launch_wator_cell_link},
    {"wator.link", sizeof(smmo_wator_args), launch_wator_link},
    {"spring_pi.force", sizeof(smmo_spring_pi_args), launch_spring_pi_force},
    {"spring_pi.node_update", sizeof(smmo_spring_pi_args), launch_spring_pi_node_update},
    {"spring_pi.link", sizeof(smmo_spring_pi_args), launch_spring_pi_link},
    {"generation.cell_count", sizeof(smmo_generation_args), launch_generation_cell_count},
    {"generation.cell_birth", sizeof(smmo_generation_args), launch_generation_cell_birth},
    {"generation.alive_update", sizeof(smmo_generation_args), launch_generation_alive_update},
    {"structure.pull", sizeof(smmo_structure_args), launch_structure_pull},
    {"structure.force", sizeof(smmo_structure_args), launch_structure_force},
    {"structure.node_update", sizeof(smmo_structure_args), launch_structure_node_update},
    {"structure.bfs_init", sizeof(smmo_structure_args), launch_structure_bfs_init, kFamilyLaunch},
    {"structure.bfs_visit", sizeof(smmo_structure_args), launch_structure_bfs_visit, kFamilyLaunch},
    {"structure.bfs_mark", sizeof(smmo_structure_args), launch_structure_bfs_mark, kFamilyLaunch},
    {"structure.bfs_delete", sizeof(smmo_structure_args), launch_structure_bfs_delete},
    {"structure.link", sizeof(smmo_structure_args), launch_structure_link},
    {"gol.generation", sizeof(smmo_gol_args), launch_gol_generation},
};
} // namespace

const MethodEntry *method_table(uint32_t *count)
{
    *count = (uint32_t)(sizeof(kMethods) / sizeof(kMethods[0]));
    return kMethods;
}

} // namespace smmo
