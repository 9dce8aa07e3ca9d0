"""Summarise a rocprofv3 rocpd database by kernel and launch shape.

usage: python -m paper_2607_20728_amd.profsummary <results.db> [rows]
"""
import sqlite3, collections, sys, re
db=sys.argv[1]
con=sqlite3.connect(db); cur=con.cursor()
rows=cur.execute("select name, grid_x, workgroup_x, lds_size, vgpr_count, accum_vgpr_count, duration from kernels").fetchall()
g=collections.defaultdict(list)
for n,gx,wx,lds,vg,ag,du in rows:
    m=re.search(r'(k_[a-z_0-9]+(<[^>]*>)?|__amd_rocclr_\w+)', n); short=m.group(1) if m else n[:40]
    g[(short,gx,lds,vg,ag)].append(du)
tot=sum(sum(v) for v in g.values())
print(f"{'kernel':28s} {'grid_x':>10s} {'lds':>6s} {'vgpr':>4s} {'agpr':>4s} {'calls':>6s} {'avg_us':>10s} {'tot_ms':>9s} {'%':>5s}")
for k,v in sorted(g.items(), key=lambda kv:-sum(kv[1]))[:int(sys.argv[2]) if len(sys.argv)>2 else 30]:
    print(f"{k[0]:28s} {k[1]:10d} {k[2]:6d} {k[3]:4d} {k[4]:4d} {len(v):6d} {sum(v)/len(v)/1e3:10.1f} {sum(v)/1e6:9.1f} {100*sum(v)/tot:5.1f}")
